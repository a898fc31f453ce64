// Analog random-walk cell transmission for gfx950 (paper: section "Monte Carlo Method",
// eq. 4 flight lengths, implicit capture of eqs. 5-6) and the standalone exit decoder.
//
// The walk has a heavy-tailed cost (mean 1 + pi tau_s / 4 flights, a long tail of diffusive
// walks), so lanes are not bound to particles: the kernel is persistent, each lane walks one
// particle at a time, and after every flight the lanes whose particle has left the cell are
// refilled from a global work counter with one atomic per wave (ballot of the idle lanes,
// mbcnt for each lane's rank among them).  The queue keeps every lane busy until it runs dry.
#include "gmc_device.hpp"
#include "gmc_internal.hpp"

namespace gmc {
namespace {

__device__ __forceinline__ int lane_rank(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(256) void walk_kernel(WalkParams p)
{
    const int lane = threadIdx.x & 63;
    const float kInf = __builtin_inff();

    bool alive = false;
    bool exhausted = false;     // wave-uniform: the work counter has passed n
    int64_t idx = 0;
    float x = 0.f, y = 0.f, u = 1.f, v = 0.f, len = 0.f, inv_sig = 0.f, cs = 0.f;
    bool scatter = false;
    uint32_t flight = 0, ncoll = 0;
    const bool analog = (p.mode == 1);

    for (;;) {
        const bool need = !alive && !exhausted;
        const uint64_t needmask = __ballot(need);
        if (needmask) {
            const int cnt = __popcll(needmask);
            const int leader = __ffsll((unsigned long long)needmask) - 1;
            unsigned long long b = 0;
            if (lane == leader) b = atomicAdd(p.queue, (unsigned long long)cnt);
            const unsigned long long base = (unsigned long long)__shfl((long long)b, leader);
            if (need) {
                const int64_t i = (int64_t)(base + (unsigned long long)lane_rank(needmask));
                if (i < p.n) {
                    idx = i;
                    const float tau = expf(p.log_tau[i]);
                    cs = p.c[i];
                    const float sig = analog ? tau : cs * tau;
                    scatter = sig > 1e-30f;      // below this 1/sig would overflow
                    inv_sig = scatter ? 1.0f / sig : 0.0f;
                    const float s = p.sin_th[i];
                    x = 0.0f;
                    y = p.y_in[i];
                    u = sqrtf(fmaxf(1.0f - s * s, 0.0f));
                    v = s;
                    len = 0.0f;
                    flight = 0;
                    ncoll = 0;
                    alive = true;
                }
            }
            if (base + (unsigned long long)cnt >= (unsigned long long)p.n) exhausted = true;
        }
        if (!__ballot(alive)) {
            if (exhausted) break;
            continue;
        }
        if (!alive) continue;

        // one flight (eq. 4): distance to the cell boundary, sampled flight, scatter or leave
        float tx = kInf, ty = kInf;
        if (u > 0.0f) tx = (1.0f - x) * fast_rcp(u);
        else if (u < 0.0f) tx = -x * fast_rcp(u);
        if (v > 0.0f) ty = (1.0f - y) * fast_rcp(v);
        else if (v < 0.0f) ty = -y * fast_rcp(v);
        const bool xface = tx <= ty;
        const float db = fmaxf(xface ? tx : ty, 0.0f);
        const U4 r = draw4(p.seed, p.id_base + (uint64_t)idx, flight, kTagWalk);
        const float ds = scatter ? neg_log(u01(r.a)) * inv_sig : kInf;
        int face = -3;   // still inside
        float pos = 0.0f;
        if (ds >= db) {
            len += db;
            if (xface) {
                const float ye = fminf(fmaxf(y + db * v, 0.0f), 1.0f);
                face = u > 0.0f ? 1 : 3;
                pos = u > 0.0f ? ye : 1.0f - ye;
            } else {
                const float xe = fminf(fmaxf(x + db * u, 0.0f), 1.0f);
                face = v > 0.0f ? 2 : 0;
                pos = v > 0.0f ? 1.0f - xe : xe;
            }
        } else {
            x += ds * u;
            y += ds * v;
            len += ds;
            ncoll += 1;
            if (analog && u01(r.c) > cs) {
                face = -1;   // absorbed at this collision
            } else {
                const float ph = u01(r.b);
                u = cos_turns(ph);
                v = sin_turns(ph);
            }
        }
        flight += 1;
        if (face == -3 && flight >= kMaxFlights) face = -2;
        if (face != -3) {
            p.face[idx] = face;
            p.pos[idx] = pos;
            p.dcos[idx] = u;
            p.dsin[idx] = v;
            p.path[idx] = len;
            if (p.ncoll) p.ncoll[idx] = ncoll;
            alive = false;
        }
    }
}

__global__ void zero_u64_kernel(unsigned long long *q) { *q = 0ull; }

__global__ __launch_bounds__(256) void decode_kernel(const float *__restrict__ raw, int64_t n,
                                                     int32_t *face, float *pos, float *dcos,
                                                     float *dsin, float *path, int32_t *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Exit e;
    const int f = decode_exit(raw[i], raw[n + i], raw[2 * n + i], raw[3 * n + i], raw[4 * n + i], e);
    face[i] = e.face;
    pos[i] = e.pos;
    dcos[i] = e.u;
    dsin[i] = e.v;
    path[i] = e.path;
    if (flags) flags[i] = f;
}

}  // namespace

hipError_t launch_walk(const WalkParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, p.queue);
    hipLaunchKernelGGL(walk_kernel, dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_decode(const float *raw, int64_t n, int32_t *face, float *pos, float *dcos,
                         float *dsin, float *path, int32_t *flags, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(decode_kernel, dim3((unsigned)blocks), dim3(256), 0, s, raw, n, face, pos,
                       dcos, dsin, path, flags);
    return hipGetLastError();
}

}  // namespace gmc
