// Cell-to-cell transport on gfx950 (paper: section "Transport Algorithm", its four stages; the
// track-length flux estimator of eqs. 5-7).
//
// A "world" holds a structure-of-arrays particle bank shared by any number of problems (each a
// grid of square cells with its own materials, source, seed and FP64 tallies), so one sampler
// launch serves particles of different problems and cells together.  One transport step:
//   gather  (stage 1)  bank -> canonical left-entry conditions, per-particle random stream ids;
//   sample  (stage 2)  the generative sampler (gmc_transmit kernels) or the analog walk;
//   apply   (stages 3-4)  FP64 rescale of the path to physical units, weight attenuation and
//            flux / absorption tallies (FP64 atomics), rotation back to the global frame, move
//            to the neighbour cell or leave / cut off, and compaction of the survivors into the
//            other bank with one atomic per wave (ballot + mbcnt).
// Volumetric births draw a source particle and take its first leg inside the birth cell with the
// analog walk or the internal (volumetric-source) model; surface-source births enter their
// boundary cell directly.
// Random numbers depend only on (problem seed, history id, cell-visit index): a history's
// result does not depend on which other problems share the bank or on its slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gmc.h"
#include "gmc_device.hpp"
#include "gmc_internal.hpp"

namespace gmc {
namespace {

struct ProblemDev {
    int32_t nx, ny;
    double L, Ly;                  // cell width (along x) and height
    float lr;                      // ln(Ly / L): 0 for square cells
    int64_t cell0;                 // first global cell index of this problem
    int32_t sx0, sy0, snx, sny;    // source block
    int32_t reflect;
    double w_min;
    uint64_t seed;
    int32_t src_face;              // -1 volumetric, else the domain side of a surface source
    int32_t xy;                    // XY geometry: directions on the sphere, projected
    uint32_t max_visits;           // a history is cut off before its cell visit of this number
};

struct BankDev {
    int32_t *cell, *pid, *entry;
    float *yin, *gx, *gy;
    double *w;
    uint32_t *hist, *event;
};

struct CellsDev {
    const double *tau, *c;         // per global cell (FP64: tallies)
    const float *ltau, *cf;        // per global cell (FP32: sampler conditions)
    double *flux, *absorbed, *leak, *cutoff;
    // path tallies per cell: sum of w_in * l_phys, sum of l_phys, number of visits; weight and
    // number of generative samples rejected by the decoder (a part of the cutoff)
    double *wpath, *path, *visits, *rej_w, *rej_n;
    const ProblemDev *prob;
};

__device__ __forceinline__ int lane_rank(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Per-workgroup tally staging: the flux, deposit and path tallies of a workgroup's particles are
// summed per cell in an LDS hash table of SLOTS slots and flushed with one FP64 global atomic
// per tally and distinct cell.
// Particles near a source crowd into few cells, whose same-address global atomics would
// otherwise serialise in L2.  A block of the one-visit-per-particle kernels holds at most 256
// particles, so at most 256 of their 512 slots fill and linear probing always ends.
template <int SLOTS>
struct TallyTable {
    static constexpr int kSlots = SLOTS;
    static constexpr int kShift = 32 - __builtin_ctz(SLOTS);   // multiplicative hash to log2(SLOTS) bits
    int32_t key[SLOTS];
    double flux[SLOTS], dep[SLOTS], wpath[SLOTS], path[SLOTS], visits[SLOTS];
};
using TallyLds = TallyTable<512>;

template <int SLOTS>
__device__ __forceinline__ void tally_init(TallyTable<SLOTS> &tl)
{
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
        tl.key[s] = -1;
        tl.flux[s] = 0.0;
        tl.dep[s] = 0.0;
        tl.wpath[s] = 0.0;
        tl.path[s] = 0.0;
        tl.visits[s] = 0.0;
    }
}

__device__ __forceinline__ void tally_add(TallyLds &tl, int cell, double phi, double dw, double wl, double l)
{
    uint32_t s = ((uint32_t)cell * 2654435761u) >> TallyLds::kShift;
    for (;;) {
        const int prev = atomicCAS(&tl.key[s], -1, cell);
        if (prev == -1 || prev == cell) break;
        s = (s + 1) & (TallyLds::kSlots - 1);
    }
    atomicAdd(&tl.flux[s], phi);
    atomicAdd(&tl.dep[s], dw);
    atomicAdd(&tl.wpath[s], wl);
    atomicAdd(&tl.path[s], l);
    atomicAdd(&tl.visits[s], 1.0);
}

template <int SLOTS>
__device__ __forceinline__ void tally_flush(TallyTable<SLOTS> &tl, const CellsDev &cd)
{
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
        const int cell = tl.key[s];
        if (cell >= 0) {
            atomicAdd(&cd.flux[cell], tl.flux[s]);
            if (tl.dep[s] != 0.0) atomicAdd(&cd.absorbed[cell], tl.dep[s]);   // 0 without absorption
            atomicAdd(&cd.wpath[cell], tl.wpath[s]);
            atomicAdd(&cd.path[cell], tl.path[s]);
            atomicAdd(&cd.visits[cell], tl.visits[s]);
        }
    }
}

// Stage 3 for one cell visit: w_out = w e^{-sigma_a l} (eq. 5), deposit dw (eq. 6) and flux
// dw / (V sigma_a) (eq. 7; w l / V when sigma_a = 0), all in FP64 with the physical path
// (path_units in units of `unit`, the length of the face the walk's frame took as its height),
// plus the path tallies w l, l and one visit, staged in the workgroup's table.
__device__ __forceinline__ double visit_tally(const CellsDev &cd, const ProblemDev &P, int cell,
                                              double w, float path_units, double unit, TallyLds &tl)
{
    const double sig_a = (1.0 - cd.c[cell]) * cd.tau[cell] / P.L;
    const double ls = (double)path_units * unit;
    const double dw = w * (-expm1(-sig_a * ls));
    const double V = P.L * P.Ly;
    const double phi = sig_a > 0.0 ? dw / (V * sig_a) : w * ls / V;
    tally_add(tl, cell, phi, dw, w * ls, ls);
    return w - dw;
}

// tally_add for a kernel whose particles may visit more distinct cells than the table holds
// (the split gather streams a particle through up to 64 cells): a cell that finds neither its
// slot nor a free one within kTallyProbes probes adds to the global tallies directly, and a
// deposit of exactly 0 (a cell without absorption) is not added.  The split gather's table has
// 1,024 slots (45 KB of LDS: its registers already hold it to three workgroups per CU).
constexpr int kTallyProbes = 4;
using TallySplit = TallyTable<1024>;
__device__ __forceinline__ void tally_add_bounded(TallySplit &tl, const CellsDev &cd, int cell, double phi,
                                                  double dw, double wl, double l)
{
    uint32_t s = ((uint32_t)cell * 2654435761u) >> TallySplit::kShift;
    for (int k = 0; k < kTallyProbes; ++k) {
        const int prev = atomicCAS(&tl.key[s], -1, cell);
        if (prev == -1 || prev == cell) {
            atomicAdd(&tl.flux[s], phi);
            if (dw != 0.0) atomicAdd(&tl.dep[s], dw);
            atomicAdd(&tl.wpath[s], wl);
            atomicAdd(&tl.path[s], l);
            atomicAdd(&tl.visits[s], 1.0);
            return;
        }
        s = (s + 1) & (TallySplit::kSlots - 1);
    }
    atomicAdd(&cd.flux[cell], phi);
    if (dw != 0.0) atomicAdd(&cd.absorbed[cell], dw);
    atomicAdd(&cd.wpath[cell], wl);
    atomicAdd(&cd.path[cell], l);
    atomicAdd(&cd.visits[cell], 1.0);
}

// visit_tally staged with tally_add_bounded.
__device__ __forceinline__ double visit_tally_bounded(const CellsDev &cd, const ProblemDev &P, int cell,
                                                      double w, float path_units, double unit, TallySplit &tl)
{
    const double sig_a = (1.0 - cd.c[cell]) * cd.tau[cell] / P.L;
    const double ls = (double)path_units * unit;
    const double dw = w * (-expm1(-sig_a * ls));
    const double V = P.L * P.Ly;
    const double phi = sig_a > 0.0 ? dw / (V * sig_a) : w * ls / V;
    tally_add_bounded(tl, cd, cell, phi, dw, w * ls, ls);
    return w - dw;
}

struct Next {
    int32_t cell, entry;
    float yin, gx, gy;
    bool alive;
};

// Stage 4: after leaving `cell` through local face `face` at counter-clockwise position pos
// with global direction (gx, gy) and weight w_out: cut off, leak, reflect or enter the
// neighbour (whose entry face is the opposite one, entered at position 1 - pos in its own
// counter-clockwise orientation, i.e. canonical height y = pos).
__device__ __forceinline__ Next move_on(const CellsDev &cd, const ProblemDev &P, int cell, int face,
                                        float pos, float gx, float gy, double w_out)
{
    Next nx{cell, 0, 0.0f, gx, gy, false};
    if (face < 0 || face > 3) {              // capped walk or rejected sample: drop its weight
        atomicAdd(&cd.cutoff[cell], w_out);  // with the cutoff
        if (face == -1) {
            atomicAdd(&cd.rej_w[cell], w_out);
            atomicAdd(&cd.rej_n[cell], 1.0);
        }
        return nx;
    }
    if (w_out < P.w_min) {
        atomicAdd(&cd.cutoff[cell], w_out);
        return nx;
    }
    const int64_t local = cell - P.cell0;
    const int ci = (int)(local % P.nx), cj = (int)(local / P.nx);
    int ni = ci, nj = cj;
    if (face == 0) nj -= 1;
    else if (face == 1) ni += 1;
    else if (face == 2) nj += 1;
    else ni -= 1;
    if (ni < 0 || nj < 0 || ni >= P.nx || nj >= P.ny) {
        if (!P.reflect) {
            atomicAdd(&cd.leak[cell], w_out);
            return nx;
        }
        nx.entry = face;                     // specular reflection back into the same cell
        nx.yin = 1.0f - pos;
        if (face == 0 || face == 2) nx.gy = -gy;
        else nx.gx = -gx;
    } else {
        nx.cell = (int32_t)(P.cell0 + (int64_t)nj * P.nx + ni);
        nx.entry = (face + 2) & 3;
        nx.yin = pos;
    }
    nx.alive = true;
    return nx;
}

// Append the alive lanes' particles to `out` (one atomic per wave) and count them per problem.
__device__ __forceinline__ void append(bool alive, const Next &nx, int32_t pid, double w,
                                       uint32_t hist, uint32_t event, BankDev out,
                                       unsigned long long *counter, unsigned long long *pcount)
{
    const int lane = threadIdx.x & 63;
    const uint64_t mask = __ballot(alive);
    if (!mask) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long b = 0;
    if (lane == leader) b = atomicAdd(counter, (unsigned long long)__popcll(mask));
    const unsigned long long base = (unsigned long long)__shfl((long long)b, leader);
    if (alive) {
        const int64_t j = (int64_t)(base + (unsigned long long)lane_rank(mask));
        out.cell[j] = nx.cell;
        out.pid[j] = pid;
        out.entry[j] = nx.entry;
        out.yin[j] = nx.yin;
        out.gx[j] = nx.gx;
        out.gy[j] = nx.gy;
        out.w[j] = w;
        out.hist[j] = hist;
        out.event[j] = event;
    }
    // per-problem alive counts: one atomic per distinct problem among the wave's survivors
    uint64_t m = mask;
    while (m) {
        const int l0 = __ffsll((unsigned long long)m) - 1;
        const int p0 = __shfl(pid, l0);
        const uint64_t same = __ballot(alive && pid == p0);
        if (lane == l0) atomicAdd(&pcount[p0], (unsigned long long)__popcll(same));
        m &= ~same;
    }
}

// Births of histories [h0, h0 + count) of problem pid: source sampling, analog first leg in the
// birth cell (global orientation), tally, move; survivors appended after the alive particles.
__global__ __launch_bounds__(256) void birth_kernel(CellsDev cd, int32_t pid, uint32_t h0,
                                                    int64_t count, BankDev out,
                                                    unsigned long long *counter,
                                                    unsigned long long *pcount)
{
    __shared__ TallyLds tl;
    tally_init(tl);
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool alive = false;
    Next nx{};
    double w_out = 0.0;
    uint32_t h = 0;
    if (t < count) {
        const ProblemDev P = cd.prob[pid];
        h = h0 + (uint32_t)t;
        const U4 r = draw4(P.seed, (uint64_t)h, 0u, kTagSource);
        const uint32_t nsrc = (uint32_t)(P.snx * P.sny);
        const uint32_t pick = __umulhi(r.a, nsrc);
        const int ci = P.sx0 + (int)(pick % (uint32_t)P.snx), cj = P.sy0 + (int)(pick / (uint32_t)P.snx);
        const int cell = (int)(P.cell0 + (int64_t)cj * P.nx + ci);
        const float ph = u01(r.d);
        // the cell's own frame [0, L / Ly] x [0, 1], lengths in units of its height Ly
        const float wa = (float)(P.L / P.Ly);
        float st = 1.0f;
        if (P.xy) {                      // isotropic on the sphere: mu from a second draw
            const U4 r2 = draw4(P.seed, (uint64_t)h, 1u, kTagSource);
            const float mu = 2.0f * u01(r2.a) - 1.0f;
            st = sqrtf(fmaxf(1.0f - mu * mu, 0.0f));
        }
        Walker W;
        walker_init(W, (float)(cd.tau[cell] * (P.Ly / P.L)), (float)cd.c[cell], 0, wa * u01_open(r.b),
                    u01_open(r.c), st * cos_turns(ph), st * sin_turns(ph), wa, P.xy != 0);
        float pos = 0.0f;
        int face;
        do {
            face = walker_flight(W, P.seed, (uint64_t)h, pos);
        } while (face == kInside);
        w_out = visit_tally(cd, P, cell, 1.0, W.len, P.Ly, tl);
        nx = move_on(cd, P, cell, face, pos, W.u, W.v, w_out);
        alive = nx.alive;
    }
    append(alive, nx, pid, w_out, h, 1u, out, counter, pcount);
    __syncthreads();
    tally_flush(tl, cd);
}

// Surface-source births of histories [h0, h0 + count): a uniformly picked cell of the source
// strip, entered through side f of the domain at a uniform canonical height with a cosine-law
// canonical direction (sin theta = 2u - 1), rotated to the global frame; no tally yet, the
// first transmission (cell visit 1) is the next transport step's.
__global__ __launch_bounds__(256) void surface_birth_kernel(CellsDev cd, int32_t pid, uint32_t h0,
                                                            int64_t count, BankDev out,
                                                            unsigned long long *counter,
                                                            unsigned long long *pcount)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool alive = false;
    Next nx{};
    uint32_t h = 0;
    if (t < count) {
        const ProblemDev P = cd.prob[pid];
        h = h0 + (uint32_t)t;
        const U4 r = draw4(P.seed, (uint64_t)h, 0u, kTagSource);
        const uint32_t nsrc = (uint32_t)(P.snx * P.sny);
        const uint32_t pick = __umulhi(r.a, nsrc);
        const int ci = P.sx0 + (int)(pick % (uint32_t)P.snx), cj = P.sy0 + (int)(pick / (uint32_t)P.snx);
        const int f = P.src_face;
        float s, cth;
        if (P.xy) {      // isotropic incident flux on the sphere: cosine sqrt(xi), azimuth psi
            const float xi = u01_open(r.c);
            cth = sqrtf(xi);
            s = sqrtf(fmaxf(1.0f - xi, 0.0f)) * cos_turns(u01(r.d));
        } else {
            s = 2.0f * u01_open(r.c) - 1.0f;
            cth = sqrtf(fmaxf(1.0f - s * s, 0.0f));
        }
        nx.cell = (int32_t)(P.cell0 + (int64_t)cj * P.nx + ci);
        nx.entry = f;
        nx.yin = u01_open(r.b);
        rot_quarter((f + 1) & 3, cth, s, nx.gx, nx.gy);
        alive = true;
    }
    append(alive, nx, pid, 1.0, h, 1u, out, counter, pcount);
}

// Source births for the generative internal model: birth cell, position and direction of
// histories [h0, h0 + count) (the same Philox draw as birth_kernel) as internal-model
// conditions in the cell's own frame; the birth event uses random stream id h.
__global__ __launch_bounds__(256) void source_kernel(CellsDev cd, int32_t pid, uint32_t h0, int64_t count,
                                                     float *ltau, float *cc, float *xb, float *yb,
                                                     float *cosb, float *sinb, uint64_t *ids, uint64_t *keys)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const ProblemDev P = cd.prob[pid];
    const uint32_t h = h0 + (uint32_t)t;
    const U4 r = draw4(P.seed, (uint64_t)h, 0u, kTagSource);
    const uint32_t nsrc = (uint32_t)(P.snx * P.sny);
    const uint32_t pick = __umulhi(r.a, nsrc);
    const int ci = P.sx0 + (int)(pick % (uint32_t)P.snx), cj = P.sy0 + (int)(pick / (uint32_t)P.snx);
    const int cell = (int)(P.cell0 + (int64_t)cj * P.nx + ci);
    const float ph = u01(r.d);
    ltau[t] = cd.ltau[cell];
    cc[t] = cd.cf[cell];
    xb[t] = u01_open(r.b);
    yb[t] = u01_open(r.c);
    cosb[t] = cos_turns(ph);
    sinb[t] = sin_turns(ph);
    ids[t] = (uint64_t)h;
    keys[t] = P.seed;
}

// Stages 3-4 of the births sampled by the internal model (exits in the cell's own frame, which
// is the global orientation): tally, move, append.
__global__ __launch_bounds__(256) void source_apply_kernel(CellsDev cd, int32_t pid, uint32_t h0,
                                                           int64_t count, const int32_t *face_c,
                                                           const float *pos, const float *dcos,
                                                           const float *dsin, const float *path,
                                                           BankDev out, unsigned long long *counter,
                                                           unsigned long long *pcount)
{
    __shared__ TallyLds tl;
    tally_init(tl);
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool alive = false;
    Next nx{};
    double w_out = 0.0;
    uint32_t h = 0;
    if (t < count) {
        const ProblemDev P = cd.prob[pid];
        h = h0 + (uint32_t)t;
        const U4 r = draw4(P.seed, (uint64_t)h, 0u, kTagSource);
        const uint32_t nsrc = (uint32_t)(P.snx * P.sny);
        const uint32_t pick = __umulhi(r.a, nsrc);
        const int ci = P.sx0 + (int)(pick % (uint32_t)P.snx), cj = P.sy0 + (int)(pick / (uint32_t)P.snx);
        const int cell = (int)(P.cell0 + (int64_t)cj * P.nx + ci);
        w_out = visit_tally(cd, P, cell, 1.0, path[t], P.L, tl);
        nx = move_on(cd, P, cell, face_c[t], pos[t], dcos[t], dsin[t], w_out);
        alive = nx.alive;
    }
    append(alive, nx, pid, w_out, h, 1u, out, counter, pcount);
    __syncthreads();
    tally_flush(tl, cd);
}

// Stage 1: canonical conditions of every alive particle.  Entry face e maps to the canonical
// left face by the rotation of k = (e + 1) mod 4 quarter turns (canonical -> local).
// The canonical cell takes the entry face as its height: left and right faces have length Ly,
// bottom and top length L, so entries through a vertical face see tau * Ly / L and aspect
// A = L / Ly, entries through a horizontal face tau and A = Ly / L.
__global__ __launch_bounds__(256) void gather_kernel(BankDev b, int64_t n_arg,
                                                     const unsigned long long *n_dev, CellsDev cd,
                                                     float *ltau, float *cc, float *yin, float *sth,
                                                     float *laspect, float *omx, uint64_t *ids,
                                                     uint64_t *keys)
{
    const int64_t n = n_dev ? (int64_t)*n_dev : n_arg;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cell = b.cell[i];
    const int e = b.entry[i];
    const int k = (e + 1) & 3;
    float U, V;
    rot_quarter((4 - k) & 3, b.gx[i], b.gy[i], U, V);
    const float lr = cd.prob[b.pid[i]].lr;
    ltau[i] = (e & 1) ? cd.ltau[cell] + lr : cd.ltau[cell];
    laspect[i] = (e & 1) ? -lr : lr;
    omx[i] = U;                          // read only in XY geometry
    cc[i] = cd.cf[cell];
    yin[i] = b.yin[i];
    sth[i] = fminf(fmaxf(V, -1.0f), 1.0f);
    ids[i] = (uint64_t)b.hist[i] | ((uint64_t)b.event[i] << 32);
    keys[i] = cd.prob[b.pid[i]].seed;
}

// Exit-record face of a particle whose history ended inside the split gather: the apply stage
// leaves it out.
constexpr int32_t kFaceEnded = -1000;

// Stage 1 with the first-flight split (models fitted on collided exits, blob flag bit 1).  Each
// particle draws its crossing's split (uncollided_exit, keyed by history and cell visit); while
// the crossings stay uncollided it is streamed through up to ff_max cells inside this kernel:
// stages 3-4 of each such crossing (FP64 attenuation and tallies, staged in the workgroup's LDS
// table with bounded probing, and the move to the neighbour) exactly as the apply stage would
// do them with the same random numbers, its bank slot then updated in place.  The crossing that ends the loop is
//   * collided: canonical conditions compacted (one atomic per wave) into the sampler's staging
//     with the bank index in sidx;
//   * the ff_max-th uncollided one: its exit record written at the particle's own index, for
//     the apply stage;
//   * one that ended the history (leak, cutoff): face kFaceEnded.
// ff_max = 1 is one crossing per particle per step.  `streamed` counts the crossings finished here.
__global__ __launch_bounds__(256) void gather_split_kernel(BankDev b, int64_t n_arg,
                                                           const unsigned long long *n_dev, CellsDev cd,
                                                           float *ltau, float *cc, float *yin, float *sth,
                                                           float *laspect, float *omx, uint64_t *ids,
                                                           uint64_t *keys, int32_t *sidx,
                                                           unsigned long long *count, int32_t *e_face,
                                                           float *e_pos, float *e_dcos, float *e_dsin,
                                                           float *e_path, int ff_max,
                                                           unsigned long long *streamed)
{
    __shared__ TallySplit tl;
    tally_init(tl);
    __syncthreads();
    const int64_t n = n_dev ? (int64_t)*n_dev : n_arg;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool collided = false;
    float lt = 0.f, c = 0.f, y = 0.f, s = 0.f, la = 0.f, ox = 0.f;
    uint64_t id = 0, key = 0;
    uint32_t nstream = 0;
    bool ended = false;
    if (i < n) {
        int cell = b.cell[i];
        int e = b.entry[i];
        float gx = b.gx[i], gy = b.gy[i], yy = b.yin[i];
        double w = b.w[i];
        uint32_t ev = b.event[i];
        const uint32_t hist = b.hist[i];
        const ProblemDev P = cd.prob[b.pid[i]];
        for (int it = 0;; ++it) {
            const int k = (e + 1) & 3;
            float U, V;
            rot_quarter((4 - k) & 3, gx, gy, U, V);
            lt = (e & 1) ? cd.ltau[cell] + P.lr : cd.ltau[cell];
            la = (e & 1) ? -P.lr : P.lr;
            c = cd.cf[cell];
            y = yy;
            s = fminf(fmaxf(V, -1.0f), 1.0f);
            ox = U;
            id = (uint64_t)hist | ((uint64_t)ev << 32);
            key = P.seed;
            const float u = P.xy ? U : sqrtf(fmaxf(1.0f - s * s, 0.0f));
            Exit ex;
            if (!uncollided_exit(expf(lt), c, y, u, s, la == 0.0f ? 1.0f : expf(la), key, id, ex)) {
                collided = true;
                break;
            }
            if (it + 1 >= ff_max) {
                e_face[i] = ex.face;
                e_pos[i] = ex.pos;
                e_dcos[i] = ex.u;
                e_dsin[i] = ex.v;
                e_path[i] = ex.path;
                break;
            }
            const double w_out = visit_tally_bounded(cd, P, cell, w, ex.path, (e & 1) ? P.Ly : P.L, tl);
            float ngx, ngy;
            rot_quarter(k, ex.u, ex.v, ngx, ngy);
            Next nx = move_on(cd, P, cell, (ex.face + k) & 3, ex.pos, ngx, ngy, w_out);
            if (nx.alive && ev + 1 >= P.max_visits) {
                atomicAdd(&cd.cutoff[cell], w_out);
                nx.alive = false;
            }
            ++nstream;
            if (!nx.alive) {
                e_face[i] = kFaceEnded;
                ended = true;
                break;
            }
            cell = nx.cell;
            e = nx.entry;
            yy = nx.yin;
            gx = nx.gx;
            gy = nx.gy;
            w = w_out;
            ++ev;
        }
        if (nstream > 0 && !ended) {
            b.cell[i] = cell;
            b.entry[i] = e;
            b.yin[i] = yy;
            b.gx[i] = gx;
            b.gy[i] = gy;
            b.w[i] = w;
            b.event[i] = ev;
        }
    }
    __syncthreads();
    tally_flush(tl, cd);
    // crossings beyond the one per particle that the step counts (a history that ended here
    // finished its step's own crossing inside the loop)
    uint32_t tot = ended ? nstream - 1 : nstream;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tot += (uint32_t)__shfl_xor((int)tot, o);
    if (lane == 0 && tot > 0) atomicAdd(streamed, (unsigned long long)tot);
    const uint64_t mask = __ballot(collided);
    if (!mask) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
    base = (unsigned long long)__shfl((long long)base, leader);
    if (collided) {
        const int64_t j = (int64_t)(base + (unsigned long long)lane_rank(mask));
        ltau[j] = lt;
        cc[j] = c;
        yin[j] = y;
        sth[j] = s;
        laspect[j] = la;
        omx[j] = ox;
        ids[j] = id;
        keys[j] = key;
        sidx[j] = (int32_t)i;
    }
}

// The sampler's exits of the compacted collided particles back to their bank indices.
__global__ __launch_bounds__(256) void scatter_kernel(int64_t n_arg, const unsigned long long *count,
                                                      const int32_t *sidx, const int32_t *f2, const float *p2,
                                                      const float *c2, const float *s2, const float *l2,
                                                      int32_t *face, float *pos, float *dcos, float *dsin,
                                                      float *path)
{
    const int64_t n = (int64_t)*count;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || j >= n_arg) return;
    const int32_t i = sidx[j];
    face[i] = f2[j];
    pos[i] = p2[j];
    dcos[i] = c2[j];
    dsin[i] = s2[j];
    path[i] = l2[j];
}

// Stages 3-4 for every alive particle, survivors compacted into `out`.
__global__ __launch_bounds__(256) void apply_kernel(BankDev in, int64_t n_arg,
                                                    const unsigned long long *n_dev, const int32_t *face_c,
                                                    const float *pos, const float *dcos,
                                                    const float *dsin, const float *path,
                                                    CellsDev cd, BankDev out,
                                                    unsigned long long *counter,
                                                    unsigned long long *pcount)
{
    __shared__ TallyLds tl;
    tally_init(tl);
    __syncthreads();
    const int64_t n = n_dev ? (int64_t)*n_dev : n_arg;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool alive = false;
    Next nx{};
    double w_out = 0.0;
    int32_t pid = 0;
    uint32_t hist = 0, event = 0;
    if (i < n && face_c[i] != kFaceEnded) {
        pid = in.pid[i];
        const ProblemDev P = cd.prob[pid];
        const int cell = in.cell[i];
        const int k = (in.entry[i] + 1) & 3;
        hist = in.hist[i];
        event = in.event[i] + 1;
        w_out = visit_tally(cd, P, cell, in.w[i], path[i], (in.entry[i] & 1) ? P.Ly : P.L, tl);
        const int fc = face_c[i];
        float gx, gy;
        rot_quarter(k, dcos[i], dsin[i], gx, gy);
        nx = move_on(cd, P, cell, fc >= 0 ? (fc + k) & 3 : fc, pos[i], gx, gy, w_out);
        if (nx.alive && event >= P.max_visits) {
            atomicAdd(&cd.cutoff[cell], w_out);
            nx.alive = false;
        }
        alive = nx.alive;
    }
    append(alive, nx, pid, w_out, hist, event, out, counter, pcount);
    __syncthreads();
    tally_flush(tl, cd);
}

__global__ void set_u64_kernel(unsigned long long *p, unsigned long long v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (i == 0) ? v : 0ull;
}

__global__ void zero_f64_kernel(double *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace
}  // namespace gmc

using namespace gmc;

struct gmc_world {
    int device = 0;
    int64_t cap = 0;
    int32_t max_problems = 0;
    int64_t max_cells = 0;
    void *mem = nullptr;
    BankDev bank[2]{};
    int cur = 0;
    int integrator = GMC_EULER;   // ODE integrator of the generative sampler
    const gmc_model *src_model = nullptr;   // internal model for births (else analog first leg)
    int src_K = 16;
    // sampler staging
    float *c_ltau = nullptr, *c_c = nullptr, *c_yin = nullptr, *c_sth = nullptr;
    float *c_x = nullptr, *c_cos = nullptr;      // internal-model births
    float *c_la = nullptr;                       // canonical ln aspect (rectangular cells)
    float *c_ox = nullptr;                       // canonical in-plane x direction (XY geometry)
    // first-flight split: bank index of each compacted collided particle, their exits, count
    int32_t *s_idx = nullptr, *s_face = nullptr;
    float *s_pos = nullptr, *s_dcos = nullptr, *s_dsin = nullptr, *s_path = nullptr;
    unsigned long long *s_count = nullptr;
    unsigned long long *n_large = nullptr;       // sampler's device-side tile choice (two count handoffs)
    unsigned long long *streamed = nullptr;      // crossings finished inside split gathers
    int ff_max = 64;                             // cells a particle may stream through per step
    int64_t stepped = 0;                         // particles stepped (one crossing each)
    uint64_t *ids = nullptr, *keys = nullptr;
    int32_t *e_face = nullptr;
    float *e_pos = nullptr, *e_dcos = nullptr, *e_dsin = nullptr, *e_path = nullptr;
    // cells and tallies
    double *tau = nullptr, *c = nullptr;
    float *ltau = nullptr, *cf = nullptr;
    double *flux = nullptr, *absorbed = nullptr, *leak = nullptr, *cutoff = nullptr;
    ProblemDev *prob = nullptr;
    unsigned long long *counters = nullptr;   // [2][1 + max_problems]: n_alive, per-problem
    unsigned long long *host_counters = nullptr;
    unsigned long long *queue = nullptr;      // the analog walk's work counter (this world's own)
    // captured transport steps, one per (sampler, model, K, integrator, bank parity, bucket)
    struct StepGraph {
        int sampler, K, integrator, cur, ff, xy;
        uint64_t model;        // serial of the model (0 for the analog walk)
        int64_t bucket;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    bool graphs = false;
    hipStream_t capture_stream = nullptr;
    std::vector<StepGraph> step_graphs;
    // host bookkeeping
    int64_t n_alive = 0;
    std::vector<int64_t> alive_pp;
    std::vector<ProblemDev> prob_host;
    std::vector<char> in_use;
    std::vector<int32_t> src_face;      // per problem slot: -1 volumetric, else a surface side
    std::vector<char> rect;             // per problem slot: non-square cells
    std::vector<char> xyg;              // per problem slot: XY geometry
    std::vector<std::pair<int64_t, int64_t>> free_cells;   // [begin, end) ranges
    std::mutex mu;

    unsigned long long *cnt(int which) { return counters + (size_t)which * (1 + max_problems); }
    double *wpath = nullptr, *path = nullptr, *visits = nullptr, *rej_w = nullptr, *rej_n = nullptr;
    CellsDev cells() const
    {
        return CellsDev{tau, c, ltau, cf, flux, absorbed, leak, cutoff, wpath, path, visits, rej_w, rej_n, prob};
    }
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte layout of one world allocation (also used to report the footprint).
struct Layout {
    size_t total = 0;
    std::vector<std::pair<void **, size_t>> parts;
    void add(void **p, size_t bytes) { parts.push_back({p, total}); total += align256(bytes); }
};

void plan(gmc_world *w, Layout &L)
{
    const size_t C = (size_t)w->cap, P = (size_t)w->max_problems, N = (size_t)w->max_cells;
    for (int b = 0; b < 2; ++b) {
        BankDev &k = w->bank[b];
        L.add((void **)&k.cell, 4 * C);
        L.add((void **)&k.pid, 4 * C);
        L.add((void **)&k.entry, 4 * C);
        L.add((void **)&k.yin, 4 * C);
        L.add((void **)&k.gx, 4 * C);
        L.add((void **)&k.gy, 4 * C);
        L.add((void **)&k.w, 8 * C);
        L.add((void **)&k.hist, 4 * C);
        L.add((void **)&k.event, 4 * C);
    }
    L.add((void **)&w->c_ltau, 4 * C);
    L.add((void **)&w->c_c, 4 * C);
    L.add((void **)&w->c_yin, 4 * C);
    L.add((void **)&w->c_sth, 4 * C);
    L.add((void **)&w->c_x, 4 * C);
    L.add((void **)&w->c_la, 4 * C);
    L.add((void **)&w->c_ox, 4 * C);
    L.add((void **)&w->s_idx, 4 * C);
    L.add((void **)&w->s_face, 4 * C);
    L.add((void **)&w->s_pos, 4 * C);
    L.add((void **)&w->s_dcos, 4 * C);
    L.add((void **)&w->s_dsin, 4 * C);
    L.add((void **)&w->s_path, 4 * C);
    L.add((void **)&w->s_count, 8);
    L.add((void **)&w->n_large, 16);
    L.add((void **)&w->streamed, 8);
    L.add((void **)&w->c_cos, 4 * C);
    L.add((void **)&w->ids, 8 * C);
    L.add((void **)&w->keys, 8 * C);
    L.add((void **)&w->e_face, 4 * C);
    L.add((void **)&w->e_pos, 4 * C);
    L.add((void **)&w->e_dcos, 4 * C);
    L.add((void **)&w->e_dsin, 4 * C);
    L.add((void **)&w->e_path, 4 * C);
    L.add((void **)&w->tau, 8 * N);
    L.add((void **)&w->c, 8 * N);
    L.add((void **)&w->ltau, 4 * N);
    L.add((void **)&w->cf, 4 * N);
    L.add((void **)&w->flux, 8 * N);
    L.add((void **)&w->absorbed, 8 * N);
    L.add((void **)&w->leak, 8 * N);
    L.add((void **)&w->cutoff, 8 * N);
    L.add((void **)&w->wpath, 8 * N);
    L.add((void **)&w->path, 8 * N);
    L.add((void **)&w->visits, 8 * N);
    L.add((void **)&w->rej_w, 8 * N);
    L.add((void **)&w->rej_n, 8 * N);
    L.add((void **)&w->prob, sizeof(ProblemDev) * P);
    L.add((void **)&w->counters, 8 * 2 * (1 + P));
    L.add((void **)&w->queue, 8);
}

int sync_counters(gmc_world *w, int which, hipStream_t s)
{
    const size_t bytes = 8 * (size_t)(1 + w->max_problems);
    hipError_t e = hipMemcpyAsync(w->host_counters, w->cnt(which), bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w->host_counters + 1 + w->max_problems, w->streamed, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "transport: reading counters");
    w->n_alive = (int64_t)w->host_counters[0];
    for (int p = 0; p < w->max_problems; ++p) w->alive_pp[p] = (int64_t)w->host_counters[1 + p];
    return GMC_OK;
}

}  // namespace

extern "C" {

int gmc_world_footprint(int64_t bank_capacity, int32_t max_problems, int64_t max_cells, size_t *bytes)
{
    if (!bytes || bank_capacity <= 0 || max_problems <= 0 || max_cells <= 0)
        return set_error(GMC_EINVAL, "gmc_world_footprint: bad argument");
    gmc_world w;
    w.cap = bank_capacity;
    w.max_problems = max_problems;
    w.max_cells = max_cells;
    Layout L;
    plan(&w, L);
    *bytes = L.total;
    return GMC_OK;
}

int gmc_world_create(int64_t bank_capacity, int32_t max_problems, int64_t max_cells, gmc_world **out)
{
    if (!out) return set_error(GMC_EINVAL, "gmc_world_create: null output");
    *out = nullptr;
    if (bank_capacity <= 0 || bank_capacity > ((int64_t)1 << 31) || max_problems <= 0 ||
        max_problems > 65536 || max_cells <= 0 || max_cells > ((int64_t)1 << 31))
        return set_error(GMC_EINVAL, "gmc_world_create: capacity out of range");
    const int irc = gmc_device_init();
    if (irc != GMC_OK) return irc;
    gmc_world *w = new gmc_world();
    w->cap = bank_capacity;
    w->max_problems = max_problems;
    w->max_cells = max_cells;
    Layout L;
    plan(w, L);
    hipError_t e = hipGetDevice(&w->device);
    if (e != hipSuccess) { delete w; return set_hip_error(e, "gmc_world_create: hipGetDevice"); }
    e = hipMalloc(&w->mem, L.total);
    if (e != hipSuccess) { delete w; return set_error(GMC_ENOMEM, "gmc_world_create: device allocation failed"); }
    for (auto &pr : L.parts) *pr.first = (char *)w->mem + pr.second;
    e = hipHostMalloc((void **)&w->host_counters, 8 * (size_t)(2 + max_problems), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(w->mem);
        delete w;
        return set_error(GMC_ENOMEM, "gmc_world_create: pinned host allocation failed");
    }
    std::memset(w->host_counters, 0, 8 * (size_t)(2 + max_problems));
    e = hipMemset(w->counters, 0, 8 * 2 * (size_t)(1 + max_problems));
    if (e == hipSuccess) e = hipMemset(w->streamed, 0, 8);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipHostFree(w->host_counters);
        (void)hipFree(w->mem);
        delete w;
        return set_hip_error(e, "gmc_world_create: clearing counters");
    }
    w->alive_pp.assign(max_problems, 0);
    w->prob_host.assign(max_problems, ProblemDev{});
    w->in_use.assign(max_problems, 0);
    w->src_face.assign(max_problems, -1);
    w->rect.assign(max_problems, 0);
    w->xyg.assign(max_problems, 0);
    w->free_cells.push_back({0, max_cells});
    *out = w;
    return GMC_OK;
}

int gmc_world_destroy(gmc_world *w)
{
    if (!w) return set_error(GMC_EINVAL, "gmc_world_destroy: null world");
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    for (auto &g : w->step_graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    if (w->capture_stream) (void)hipStreamDestroy(w->capture_stream);
    if (w->host_counters) e1 = hipHostFree(w->host_counters);
    if (w->mem) e2 = hipFree(w->mem);
    delete w;
    if (e1 != hipSuccess) return set_hip_error(e1, "gmc_world_destroy");
    if (e2 != hipSuccess) return set_hip_error(e2, "gmc_world_destroy");
    return GMC_OK;
}

int gmc_problem_add(gmc_world *w, const gmc_problem_desc *d, int32_t *pid_out, void *stream)
{
    if (!w || !d || !pid_out) return set_error(GMC_EINVAL, "gmc_problem_add: null pointer");
    if (d->nx <= 0 || d->ny <= 0 || !(d->L > 0.0) || !d->tau || !d->c)
        return set_error(GMC_EINVAL, "gmc_problem_add: bad grid or materials");
    if (d->src_nx <= 0 || d->src_ny <= 0 || d->src_x0 < 0 || d->src_y0 < 0 ||
        d->src_x0 + d->src_nx > d->nx || d->src_y0 + d->src_ny > d->ny)
        return set_error(GMC_EINVAL, "gmc_problem_add: source block outside the grid");
    if (!(d->Ly >= 0.0) || !std::isfinite(d->Ly))
        return set_error(GMC_EINVAL, "gmc_problem_add: Ly must be 0 (square cells) or positive");
    const double Ly = d->Ly > 0.0 ? d->Ly : d->L;
    if (d->xy != 0 && d->xy != 1)
        return set_error(GMC_EINVAL, "gmc_problem_add: xy must be 0 (flatland) or 1 (XY geometry)");
    if (d->max_visits != 0 && (d->max_visits < 2 || d->max_visits > ((int64_t)1 << 31)))
        return set_error(GMC_EINVAL, "gmc_problem_add: max_visits must be 0 (2^24) or in 2..2^31");
    if (d->src_face < -1 || d->src_face > 3)
        return set_error(GMC_EINVAL, "gmc_problem_add: src_face must be -1 (volumetric) or a side 0..3");
    if (d->src_face >= 0) {
        const int f = d->src_face;
        const bool strip = (f == 3) ? (d->src_x0 == 0 && d->src_nx == 1)
                         : (f == 1) ? (d->src_x0 == d->nx - 1 && d->src_nx == 1)
                         : (f == 0) ? (d->src_y0 == 0 && d->src_ny == 1)
                                    : (d->src_y0 == d->ny - 1 && d->src_ny == 1);
        if (!strip || d->reflect)
            return set_error(GMC_EINVAL, "gmc_problem_add: a surface source needs a one-cell strip "
                                         "along its side of the domain and vacuum boundaries");
    }
    const int64_t n = (int64_t)d->nx * d->ny;
    for (int64_t i = 0; i < n; ++i)
        if (!(d->tau[i] >= 0.0) || !std::isfinite(d->tau[i]) || !(d->c[i] >= 0.0) || !(d->c[i] <= 1.0))
            return set_error(GMC_EINVAL, "gmc_problem_add: tau must be finite >= 0 and c in [0, 1]");
    std::lock_guard<std::mutex> lk(w->mu);
    for (int q = 0; q < w->max_problems; ++q)
        if (w->in_use[q] && w->xyg[q] != (d->xy ? 1 : 0))
            return set_error(GMC_EINVAL, "gmc_problem_add: the world's problems share one geometry (flatland or XY)");
    int pid = -1;
    for (int p = 0; p < w->max_problems; ++p)
        if (!w->in_use[p]) { pid = p; break; }
    if (pid < 0) return set_error(GMC_ENOMEM, "gmc_problem_add: no free problem slot");
    int64_t cell0 = -1;
    for (auto &r : w->free_cells)
        if (r.second - r.first >= n) {
            cell0 = r.first;
            r.first += n;
            break;
        }
    if (cell0 < 0) return set_error(GMC_ENOMEM, "gmc_problem_add: no room for the cells");
    w->free_cells.erase(std::remove_if(w->free_cells.begin(), w->free_cells.end(),
                                       [](const std::pair<int64_t, int64_t> &r) { return r.first >= r.second; }),
                        w->free_cells.end());
    std::vector<float> lt(n), cf(n);
    for (int64_t i = 0; i < n; ++i) {
        lt[i] = d->tau[i] > 0.0 ? (float)std::log(d->tau[i]) : -1.0e4f;
        cf[i] = (float)d->c[i];
    }
    const uint32_t max_visits = d->max_visits == 0 ? (1u << 24) : (uint32_t)d->max_visits;
    ProblemDev P{d->nx, d->ny, d->L, Ly, (float)std::log(Ly / d->L), cell0, d->src_x0, d->src_y0,
                 d->src_nx, d->src_ny, d->reflect ? 1 : 0, d->w_min, d->seed, d->src_face, d->xy ? 1 : 0,
                 max_visits};
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(w->tau + cell0, d->tau, 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w->c + cell0, d->c, 8 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w->ltau + cell0, lt.data(), 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w->cf + cell0, cf.data(), 4 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w->prob + pid, &P, sizeof P, hipMemcpyHostToDevice, s);
    double *tallies[9] = {w->flux, w->absorbed, w->leak, w->cutoff, w->wpath, w->path, w->visits, w->rej_w, w->rej_n};
    for (double *t : tallies) {
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks_for(n)), dim3(256), 0, s, t + cell0, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);      // the host staging vectors go away
    if (e != hipSuccess) {
        w->free_cells.push_back({cell0, cell0 + n});
        return set_hip_error(e, "gmc_problem_add: upload");
    }
    w->in_use[pid] = 1;
    w->src_face[pid] = d->src_face;
    w->rect[pid] = Ly != d->L;
    w->xyg[pid] = d->xy ? 1 : 0;
    w->prob_host[pid] = P;
    w->alive_pp[pid] = 0;
    *pid_out = pid;
    return GMC_OK;
}

int gmc_problem_remove(gmc_world *w, int32_t pid)
{
    if (!w || pid < 0 || pid >= (w ? w->max_problems : 0) || !w->in_use[pid])
        return set_error(GMC_EINVAL, "gmc_problem_remove: no such problem");
    std::lock_guard<std::mutex> lk(w->mu);
    if (w->alive_pp[pid] != 0)
        return set_error(GMC_EINVAL, "gmc_problem_remove: the problem still has particles in flight");
    const ProblemDev &P = w->prob_host[pid];
    w->free_cells.push_back({P.cell0, P.cell0 + (int64_t)P.nx * P.ny});
    std::sort(w->free_cells.begin(), w->free_cells.end());
    std::vector<std::pair<int64_t, int64_t>> merged;
    for (auto &r : w->free_cells) {
        if (!merged.empty() && merged.back().second >= r.first) merged.back().second = std::max(merged.back().second, r.second);
        else merged.push_back(r);
    }
    w->free_cells.swap(merged);
    w->in_use[pid] = 0;
    w->rect[pid] = 0;
    w->xyg[pid] = 0;
    return GMC_OK;
}

int gmc_world_inject(gmc_world *w, int32_t pid, uint64_t h_begin, int64_t count, void *stream,
                     int64_t *n_alive_out)
{
    if (!w || pid < 0 || pid >= w->max_problems || !w->in_use[pid])
        return set_error(GMC_EINVAL, "gmc_world_inject: no such problem");
    if (count < 0 || h_begin + (uint64_t)count > ((uint64_t)1 << 32))
        return set_error(GMC_EINVAL, "gmc_world_inject: history ids must stay below 2^32");
    if (count > w->cap - w->n_alive)
        return set_error(GMC_ENOMEM, "gmc_world_inject: not enough free bank slots");
    if (w->src_face[pid] < 0 && w->src_model && (w->rect[pid] || w->xyg[pid]))
        return set_error(GMC_EINVAL, "gmc_world_inject: the internal model serves flatland square cells only");
    hipStream_t s = (hipStream_t)stream;
    if (count > 0) {
        const int which = w->cur;
        unsigned long long *ctr = w->cnt(which);
        // the bank's particle counter restarts at the number alive; per-problem counts continue
        hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(1), 0, s, ctr, (unsigned long long)w->n_alive, 1);
        if (w->src_face[pid] >= 0) {
            hipLaunchKernelGGL(surface_birth_kernel, dim3(blocks_for(count)), dim3(256), 0, s, w->cells(),
                               pid, (uint32_t)h_begin, count, w->bank[which], ctr, ctr + 1);
        } else if (!w->src_model) {
            hipLaunchKernelGGL(birth_kernel, dim3(blocks_for(count)), dim3(256), 0, s, w->cells(), pid,
                               (uint32_t)h_begin, count, w->bank[which], ctr, ctr + 1);
        } else {
            hipLaunchKernelGGL(source_kernel, dim3(blocks_for(count)), dim3(256), 0, s, w->cells(), pid,
                               (uint32_t)h_begin, count, w->c_ltau, w->c_c, w->c_x, w->c_yin, w->c_cos,
                               w->c_sth, w->ids, w->keys);
            const gmc_model *m = w->src_model;
            MlpParams p = m->tmpl;
            p.log_tau = w->c_ltau;
            p.c = w->c_c;
            p.x_in = w->c_x;
            p.y_in = w->c_yin;
            p.cos_phi = w->c_cos;
            p.sin_th = w->c_sth;
            p.noise = nullptr;
            p.raw = nullptr;
            p.ids = w->ids;
            p.keys = w->keys;
            p.face = w->e_face;
            p.pos = w->e_pos;
            p.dcos = w->e_dcos;
            p.dsin = w->e_dsin;
            p.path = w->e_path;
            p.n = count;
            p.n_dev = nullptr;
            p.K = w->src_K;
            p.integrator = w->integrator;
            p.seed = 0;
            p.id_base = 0;
            const int cu = device_cu_count();
            if (cu <= 0) return set_error(GMC_EDEVICE, "gmc_world_inject: cannot query the device");
            hipError_t e = launch_mlp_ode(m->precision, m->hidden, p, cu, s);
            if (e != hipSuccess) return set_hip_error(e, "gmc_world_inject: internal sampler");
            hipLaunchKernelGGL(source_apply_kernel, dim3(blocks_for(count)), dim3(256), 0, s, w->cells(), pid,
                               (uint32_t)h_begin, count, w->e_face, w->e_pos, w->e_dcos, w->e_dsin,
                               w->e_path, w->bank[which], ctr, ctr + 1);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return set_hip_error(e, "gmc_world_inject: launch");
        const int rc = sync_counters(w, which, s);
        if (rc != GMC_OK) return rc;
    }
    if (n_alive_out) *n_alive_out = w->n_alive;
    return GMC_OK;
}

int gmc_world_set_source_model(gmc_world *w, const gmc_model *m, int K)
{
    if (!w) return set_error(GMC_EINVAL, "gmc_world_set_source_model: null world");
    if (m && (m->n_in != 12 || K < 1 || K > 1024))
        return set_error(GMC_EINVAL, "gmc_world_set_source_model: needs an internal model (12 inputs) and K in 1..1024");
    std::lock_guard<std::mutex> lk(w->mu);
    w->src_model = m;
    w->src_K = K;
    return GMC_OK;
}

int gmc_world_set_integrator(gmc_world *w, int integrator)
{
    if (!w) return set_error(GMC_EINVAL, "gmc_world_set_integrator: null world");
    if (integrator != GMC_EULER && integrator != GMC_RK4)
        return set_error(GMC_EINVAL, "gmc_world_set_integrator: integrator must be GMC_EULER or GMC_RK4");
    std::lock_guard<std::mutex> lk(w->mu);
    w->integrator = integrator;
    return GMC_OK;
}

int gmc_world_set_streaming(gmc_world *w, int max_crossings)
{
    if (!w) return set_error(GMC_EINVAL, "gmc_world_set_streaming: null world");
    if (max_crossings < 1 || max_crossings > 1024)
        return set_error(GMC_EINVAL, "gmc_world_set_streaming: max_crossings must be in 1..1024");
    std::lock_guard<std::mutex> lk(w->mu);
    w->ff_max = max_crossings;
    return GMC_OK;
}

int gmc_world_transmissions(const gmc_world *w, int64_t *count)
{
    if (!w || !count) return set_error(GMC_EINVAL, "gmc_world_transmissions: null argument");
    *count = w->stepped + (int64_t)w->host_counters[1 + w->max_problems];
    return GMC_OK;
}

int gmc_world_set_graphs(gmc_world *w, int enable)
{
    if (!w) return set_error(GMC_EINVAL, "gmc_world_set_graphs: null world");
    std::lock_guard<std::mutex> lk(w->mu);
    if (enable && !w->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&w->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            w->capture_stream = nullptr;
            return set_hip_error(e, "gmc_world_set_graphs: capture stream");
        }
    }
    w->graphs = enable != 0;
    return GMC_OK;
}

namespace {

// XY geometry of the world's problems (they all share one geometry)
bool world_xy(const gmc_world *w)
{
    for (int p = 0; p < w->max_problems; ++p)
        if (w->in_use[p] && w->xyg[p]) return true;
    return false;
}

// Enqueue one transport step on `s`: gather, sampler, counter reset, apply.  Grids are sized for
// `n_launch` particles; the kernels process n_dev[0] of them when n_dev is given (a captured step
// serves every count up to its bucket), else n_launch.
int enqueue_step(gmc_world *w, int sampler, const gmc_model *m, int K, hipStream_t s, int64_t n_launch,
                 const unsigned long long *n_dev)
{
    const int cur = w->cur, nxt = 1 - cur;
    const bool split = sampler == GMC_SAMPLER_GMC && m->collided;
    if (split) {
        hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(1), 0, s, w->s_count, 0ull, 1);
        hipLaunchKernelGGL(gather_split_kernel, dim3(blocks_for(n_launch)), dim3(256), 0, s, w->bank[cur],
                           n_launch, n_dev, w->cells(), w->c_ltau, w->c_c, w->c_yin, w->c_sth, w->c_la,
                           w->c_ox, w->ids, w->keys, w->s_idx, w->s_count, w->e_face, w->e_pos, w->e_dcos,
                           w->e_dsin, w->e_path, w->ff_max, w->streamed);
    } else {
        hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n_launch)), dim3(256), 0, s, w->bank[cur], n_launch,
                           n_dev, w->cells(), w->c_ltau, w->c_c, w->c_yin, w->c_sth, w->c_la, w->c_ox, w->ids,
                           w->keys);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "gmc_transport_step: gather");
    const int cu = device_cu_count();
    if (cu <= 0) return set_error(GMC_EDEVICE, "gmc_transport_step: cannot query the device");
    if (sampler == GMC_SAMPLER_GMC) {
        MlpParams p = m->tmpl;
        p.log_tau = w->c_ltau;
        p.c = w->c_c;
        p.y_in = w->c_yin;
        p.sin_th = w->c_sth;
        p.log_aspect = (m->n_in == 11 && !m->xy) ? w->c_la : nullptr;
        p.omega_x = m->xy ? w->c_ox : nullptr;
        p.noise = nullptr;
        p.raw = nullptr;
        p.ids = w->ids;
        p.keys = w->keys;
        p.face = split ? w->s_face : w->e_face;
        p.pos = split ? w->s_pos : w->e_pos;
        p.dcos = split ? w->s_dcos : w->e_dcos;
        p.dsin = split ? w->s_dsin : w->e_dsin;
        p.path = split ? w->s_path : w->e_path;
        p.n = n_launch;
        p.n_dev = split ? w->s_count : n_dev;
        p.n_dev_large = p.n_dev ? w->n_large : nullptr;
        p.K = K;
        p.integrator = w->integrator;
        p.seed = 0;
        p.id_base = 0;
        e = launch_mlp_ode(m->precision, m->hidden, p, cu, s);
        if (e == hipSuccess && split) {
            hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(n_launch)), dim3(256), 0, s, n_launch, w->s_count,
                               w->s_idx, w->s_face, w->s_pos, w->s_dcos, w->s_dsin, w->s_path, w->e_face,
                               w->e_pos, w->e_dcos, w->e_dsin, w->e_path);
            e = hipGetLastError();
        }
    } else {
        WalkParams p{};
        p.log_tau = w->c_ltau;
        p.c = w->c_c;
        p.y_in = w->c_yin;
        p.sin_th = w->c_sth;
        p.log_aspect = w->c_la;
        p.omega_x = world_xy(w) ? w->c_ox : nullptr;
        p.face = w->e_face;
        p.pos = w->e_pos;
        p.dcos = w->e_dcos;
        p.dsin = w->e_dsin;
        p.path = w->e_path;
        p.ncoll = nullptr;
        p.ids = w->ids;
        p.keys = w->keys;
        p.n = n_launch;
        p.n_dev = n_dev;
        p.mode = GMC_MODE_CONTINUOUS;
        p.queue = w->queue;
        e = launch_walk(p, walk_grid(n_launch, cu), s);
    }
    if (e != hipSuccess) return set_hip_error(e, "gmc_transport_step: sampler");
    unsigned long long *ctr = w->cnt(nxt);
    hipLaunchKernelGGL(set_u64_kernel, dim3(blocks_for(1 + w->max_problems)), dim3(256), 0, s,
                       ctr, 0ull, 1 + w->max_problems);
    hipLaunchKernelGGL(apply_kernel, dim3(blocks_for(n_launch)), dim3(256), 0, s, w->bank[cur], n_launch,
                       n_dev, w->e_face, w->e_pos, w->e_dcos, w->e_dsin, w->e_path, w->cells(),
                       w->bank[nxt], ctr, ctr + 1);
    e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "gmc_transport_step: apply");
    return GMC_OK;
}

// Bucket of a particle count: the next power of two (at least 1024), capped at the capacity.
int64_t step_bucket(const gmc_world *w, int64_t n)
{
    int64_t b = 1024;
    while (b < n) b <<= 1;
    return std::min<int64_t>(b, w->cap);
}

// The captured step for this configuration and bucket, captured (and instantiated) on first use.
// The captured kernels read the particle count from the current bank's device counter.
int step_graph(gmc_world *w, int sampler, const gmc_model *m, int K, int64_t bucket, hipGraphExec_t *exec)
{
    const int integ = (sampler == GMC_SAMPLER_GMC) ? w->integrator : 0;
    const uint64_t mm = (sampler == GMC_SAMPLER_GMC) ? m->serial : 0;
    const int KK = (sampler == GMC_SAMPLER_GMC) ? K : 0;
    const int ff = (sampler == GMC_SAMPLER_GMC && m->collided) ? w->ff_max : 0;
    // the captured launches bake in the world's geometry (the analog walk reads omega_x only in
    // XY geometry), so the key holds it too
    const int xy = world_xy(w) ? 1 : 0;
    for (auto &g : w->step_graphs)
        if (g.sampler == sampler && g.model == mm && g.K == KK && g.integrator == integ && g.cur == w->cur &&
            g.ff == ff && g.xy == xy && g.bucket == bucket) {
            *exec = g.exec;
            return GMC_OK;
        }
    hipStream_t cs = w->capture_stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return set_hip_error(e, "gmc_transport_step: begin capture");
    const int rc = enqueue_step(w, sampler, m, K, cs, bucket, w->cnt(w->cur));
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rc != GMC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return set_hip_error(e, "gmc_transport_step: end capture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return set_hip_error(e, "gmc_transport_step: instantiate");
    }
    w->step_graphs.push_back({sampler, KK, integ, w->cur, ff, xy, mm, bucket, graph, x});
    *exec = x;
    return GMC_OK;
}

}  // namespace

int gmc_transport_step(gmc_world *w, int sampler, const gmc_model *m, int K, void *stream,
                       int64_t *n_alive_out)
{
    if (!w) return set_error(GMC_EINVAL, "gmc_transport_step: null world");
    if (sampler != GMC_SAMPLER_GMC && sampler != GMC_SAMPLER_MC)
        return set_error(GMC_EINVAL, "gmc_transport_step: sampler must be GMC or MC");
    if (sampler == GMC_SAMPLER_GMC && (!m || K < 1 || K > 1024))
        return set_error(GMC_EINVAL, "gmc_transport_step: GMC needs a model and K in 1..1024");
    if (sampler == GMC_SAMPLER_GMC && m->n_in != 10 && m->n_in != 11)
        return set_error(GMC_EINVAL, "gmc_transport_step: the model is not a boundary model (10 or 11 inputs)");
    if (sampler == GMC_SAMPLER_GMC && m->n_in == 10 &&
        std::any_of(w->rect.begin(), w->rect.end(), [](char r) { return r != 0; }))
        return set_error(GMC_EINVAL, "gmc_transport_step: rectangular cells need an 11-input boundary model");
    if (sampler == GMC_SAMPLER_GMC && world_xy(w) != m->xy)
        return set_error(GMC_EINVAL, "gmc_transport_step: the model's geometry (flatland / XY) differs from the world's");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = w->n_alive;
    if (n > 0) {
        int rc;
        if (w->graphs) {
            hipGraphExec_t x = nullptr;
            rc = step_graph(w, sampler, m, K, step_bucket(w, n), &x);
            if (rc != GMC_OK) return rc;
            const hipError_t e = hipGraphLaunch(x, s);
            if (e != hipSuccess) return set_hip_error(e, "gmc_transport_step: graph launch");
        } else {
            rc = enqueue_step(w, sampler, m, K, s, n, nullptr);
            if (rc != GMC_OK) return rc;
        }
        const int nxt = 1 - w->cur;
        w->cur = nxt;
        w->stepped += n;
        rc = sync_counters(w, nxt, s);
        if (rc != GMC_OK) return rc;
    }
    if (n_alive_out) *n_alive_out = w->n_alive;
    return GMC_OK;
}

int gmc_problem_alive(const gmc_world *w, int32_t pid, int64_t *n_alive)
{
    if (!w || !n_alive || pid < 0 || pid >= w->max_problems || !w->in_use[pid])
        return set_error(GMC_EINVAL, "gmc_problem_alive: no such problem");
    *n_alive = w->alive_pp[pid];
    return GMC_OK;
}

int gmc_problem_tally(gmc_world *w, int32_t pid, double *flux, double *absorbed, double *leak,
                      double *cutoff, void *stream)
{
    if (!w || pid < 0 || pid >= w->max_problems || !w->in_use[pid])
        return set_error(GMC_EINVAL, "gmc_problem_tally: no such problem");
    const ProblemDev &P = w->prob_host[pid];
    const int64_t n = (int64_t)P.nx * P.ny;
    hipStream_t s = (hipStream_t)stream;
    double *dst[4] = {flux, absorbed, leak, cutoff};
    const double *src[4] = {w->flux, w->absorbed, w->leak, w->cutoff};
    hipError_t e = hipSuccess;
    for (int t = 0; t < 4 && e == hipSuccess; ++t)
        if (dst[t]) e = hipMemcpyAsync(dst[t], src[t] + P.cell0, 8 * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "gmc_problem_tally: copy");
    return GMC_OK;
}

int gmc_problem_path_tally(gmc_world *w, int32_t pid, double *wpath, double *path, double *visits,
                           double *rejected_w, double *rejected_n, void *stream)
{
    if (!w || pid < 0 || pid >= w->max_problems || !w->in_use[pid])
        return set_error(GMC_EINVAL, "gmc_problem_path_tally: no such problem");
    const ProblemDev &P = w->prob_host[pid];
    const int64_t n = (int64_t)P.nx * P.ny;
    hipStream_t s = (hipStream_t)stream;
    double *dst[5] = {wpath, path, visits, rejected_w, rejected_n};
    const double *src[5] = {w->wpath, w->path, w->visits, w->rej_w, w->rej_n};
    hipError_t e = hipSuccess;
    for (int t = 0; t < 5 && e == hipSuccess; ++t)
        if (dst[t]) e = hipMemcpyAsync(dst[t], src[t] + P.cell0, 8 * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "gmc_problem_path_tally: copy");
    return GMC_OK;
}

}  // extern "C"
