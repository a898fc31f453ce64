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
    bool alive = false;
    bool exhausted = false;     // wave-uniform: the work counter has passed n
    int64_t idx = 0;
    uint64_t key = p.seed, stream = 0;
    Walker w;
    walker_init(w, 0.0f, 0.0f, 0, 0.0f, 0.0f, 1.0f, 0.0f);
    const int64_t n = p.n_dev ? (int64_t)*p.n_dev : p.n;

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
                if (i < n) {
                    idx = i;
                    const float s = p.sin_th[i];
                    const float la = p.log_aspect ? p.log_aspect[i] : 0.0f;
                    const float wa = la == 0.0f ? 1.0f : expf(la);
                    if (p.x_in) {       // birth inside the cell
                        walker_init(w, expf(p.log_tau[i]), p.c[i], p.mode, p.x_in[i], p.y_in[i],
                                    p.cos_phi[i], s, wa);
                    } else {            // entry on the left face
                        walker_init(w, expf(p.log_tau[i]), p.c[i], p.mode, 0.0f, p.y_in[i],
                                    sqrtf(fmaxf(1.0f - s * s, 0.0f)), s, wa);
                    }
                    stream = p.ids ? p.ids[i] : p.id_base + (uint64_t)i;
                    key = p.keys ? p.keys[i] : p.seed;
                    alive = true;
                }
            }
            if (base + (unsigned long long)cnt >= (unsigned long long)n) exhausted = true;
        }
        if (!__ballot(alive)) {
            if (exhausted) break;
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

hipError_t launch_decode(const float *raw, int64_t n, int32_t *face, float *pos, float *dcos,
                         float *dsin, float *path, int32_t *flags, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(decode_kernel, dim3((unsigned)blocks), dim3(256), 0, s, raw, n, face, pos,
                       dcos, dsin, path, flags);
    return hipGetLastError();
}

}  // namespace gmc
