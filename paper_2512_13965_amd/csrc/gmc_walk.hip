// Analog random-walk cell transmission for gfx950 (paper: section "Monte Carlo Method",
// eq. 4 flight lengths, implicit capture of eqs. 5-6) and the standalone exit decoder.
//
// The walk has a heavy-tailed cost (mean 1 + pi tau_s / 4 flights, a long tail of diffusive
// walks), so lanes are not bound to particles: the kernel is persistent, each lane walks one
// particle at a time, and after every flight the lanes whose particle has left the cell are
// refilled (ballot of the idle lanes, mbcnt for each lane's rank among them) from a pool of
// indices the wave holds, which it refills in chunks from a global work counter with one
// atomic.  The queue keeps every lane busy until it runs dry.
#include "gmc_device.hpp"
#include "gmc_internal.hpp"

namespace gmc {

// Work counters of the allocation-free walk: every GPU the library runs on holds this array
// until the process ends; each mc_transmit_noalloc call on a device takes the next of its
// kNoAllocCounters counters in turn and zeroes it with a kernel before the walk.
static __device__ __align__(256) unsigned long long scratch[kNoAllocCounters];

// Device address of `scratch` on the current device (each device has its own copy).  Host code
// passes this address to kernels, never the array's name.
hipError_t lookup_noalloc_counters(unsigned long long **base)
{
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    *base = e == hipSuccess ? (unsigned long long *)ptr : nullptr;
    return e;
}

namespace {

__device__ __forceinline__ int lane_rank(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(256) void walk_kernel(WalkParams p)
{
    const int lane = threadIdx.x & 63;
    bool alive = false;
    int64_t idx = 0;
    uint64_t key = p.seed, stream = 0;
    Walker w;
    walker_init(w, 0.0f, 0.0f, 0, 0.0f, 0.0f, 1.0f, 0.0f);
    const int64_t n = p.n_dev ? (int64_t)*p.n_dev : p.n;
    // Work arrives in chunks: one atomic on the global counter gives a wave `chunk` (or more)
    // consecutive particle indices, which it hands to its idle lanes over the following
    // iterations.  The counter then sees about n / chunk atomics instead of one per refill
    // (same-address atomics serialise in L2 and bound a walk whose lanes free up one at a time).
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    int64_t chunk = n / (waves * 4);
    chunk = chunk < 1 ? 1 : (chunk > 64 ? 64 : chunk);
    int64_t pool_next = 0, pool_end = 0;   // wave-uniform: unstarted indices held by this wave
    bool exhausted = false;                // wave-uniform: the global counter has reached n

    for (;;) {
        const bool need = !alive && !(exhausted && pool_next >= pool_end);
        const uint64_t needmask = __ballot(need);
        if (needmask) {
            const int64_t cnt = __popcll(needmask);
            const int64_t avail = pool_end - pool_next;
            int64_t base2 = 0, end2 = 0;
            if (avail < cnt && !exhausted) {
                const int64_t take = (cnt - avail) > chunk ? (cnt - avail) : chunk;
                const int leader = __ffsll((unsigned long long)needmask) - 1;
                unsigned long long b = 0;
                if (lane == leader) b = atomicAdd(p.queue, (unsigned long long)take);
                base2 = (int64_t)__shfl((long long)b, leader);
                end2 = base2 + take < n ? base2 + take : n;
                if (base2 + take >= n) exhausted = true;
                if (base2 > end2) base2 = end2;    // past the end: nothing left
            }
            if (need) {
                const int64_t r = lane_rank(needmask);
                int64_t i = -1;
                if (r < avail) i = pool_next + r;
                else if (base2 + (r - avail) < end2) i = base2 + (r - avail);
                if (i >= 0) {
                    idx = i;
                    const float s = p.sin_th[i];
                    const float la = p.log_aspect ? p.log_aspect[i] : 0.0f;
                    const float wa = la == 0.0f ? 1.0f : expf(la);
                    if (p.x_in) {       // birth inside the cell
                        walker_init(w, expf(p.log_tau[i]), p.c[i], p.mode, p.x_in[i], p.y_in[i],
                                    p.cos_phi[i], s, wa);
                    } else if (p.omega_x) {   // entry on the left face, XY geometry
                        walker_init(w, expf(p.log_tau[i]), p.c[i], p.mode, 0.0f, p.y_in[i],
                                    p.omega_x[i], s, wa, true);
                    } else {            // entry on the left face
                        walker_init(w, expf(p.log_tau[i]), p.c[i], p.mode, 0.0f, p.y_in[i],
                                    sqrtf(fmaxf(1.0f - s * s, 0.0f)), s, wa);
                    }
                    stream = p.ids ? p.ids[i] : p.id_base + (uint64_t)i;
                    key = p.keys ? p.keys[i] : p.seed;
                    alive = true;
                }
            }
            if (avail >= cnt) {
                pool_next += cnt;
            } else {                  // old pool used up; the rest of the new chunk remains
                const int64_t used = cnt - avail;
                pool_next = base2 + used < end2 ? base2 + used : end2;
                pool_end = end2;
            }
        }
        if (!__ballot(alive)) {
            if (exhausted && pool_next >= pool_end) break;
            continue;
        }
        if (!alive) continue;

        float pos = 0.0f;
        const int face = walker_flight(w, key, stream, pos);
        if (face != kInside) {
            p.face[idx] = face;
            p.pos[idx] = pos;
            p.dcos[idx] = w.u;
            p.dsin[idx] = w.v;
            p.path[idx] = w.len;
            if (p.ncoll) p.ncoll[idx] = w.ncoll;
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

// First-flight split of n canonical transmissions (uncollided_exit): flag[i] = 1 and the exit
// record written for an uncollided crossing, flag[i] = 0 and the record left untouched otherwise.
__global__ __launch_bounds__(256) void split_kernel(WalkParams p, int32_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const float s = p.sin_th[i];
    const float la = p.log_aspect ? p.log_aspect[i] : 0.0f;
    const float wa = la == 0.0f ? 1.0f : expf(la);
    const float u = p.omega_x ? p.omega_x[i] : sqrtf(fmaxf(1.0f - s * s, 0.0f));
    const uint64_t id = p.ids ? p.ids[i] : p.id_base + (uint64_t)i;
    const uint64_t key = p.keys ? p.keys[i] : p.seed;
    Exit e;
    const bool unc = uncollided_exit(expf(p.log_tau[i]), p.c[i], p.y_in[i], u, s, wa, key, id, e);
    flag[i] = unc ? 1 : 0;
    if (unc) {
        p.face[i] = e.face;
        p.pos[i] = e.pos;
        p.dcos[i] = e.u;
        p.dsin[i] = e.v;
        p.path[i] = e.path;
    }
}

hipError_t launch_split(const WalkParams &p, int32_t *flag, hipStream_t s)
{
    const int64_t blocks = (p.n + 255) / 256;
    hipLaunchKernelGGL(split_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, flag);
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
