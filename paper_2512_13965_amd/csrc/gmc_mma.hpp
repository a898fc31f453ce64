// Building blocks shared by the fused sampler kernels (gmc_mlp.hip: the plain velocity MLP;
// gmc_film.hip: the residual network with adaptive modulation): operand fragment loads through
// buffer resources, the 32x32 MFMA k-loop over an LDS activation tile, bias initialisation of
// accumulator tiles, the store of packed accumulator tiles into an LDS activation tile in the
// column order the next layer reads, and a sample's inputs (noise, condition features) and
// outputs (raw state, decoded exit).
#pragma once

#include <utility>

#include "gmc_device.hpp"
#include "gmc_internal.hpp"

// Weight fragments the half-range k-loop (mma_seq) loads ahead of the k-block it multiplies.
#ifndef GMC_PFA
#define GMC_PFA 2
#endif

namespace gmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

using Rsrc = __amdgpu_buffer_rsrc_t;

// Buffer resource over `bytes` bytes at p (raw, 32-bit elements): loads beyond the range return 0.
__device__ __forceinline__ Rsrc make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// 16-byte load at byte offset voff (per lane) + soff (wave-uniform) of a buffer resource.
__device__ __forceinline__ u32x4 buf_load16(Rsrc r, int voff, int soff)
{
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

template <int P>
struct Mma;

template <>
struct Mma<kF32> {
    using Frag = u32x4;
    static __device__ __forceinline__ void run(f32x16 &acc, const Frag &a, const Frag &b, int)
    {
        // reinterpret whole vectors: a bit_cast of a single vector component reads the
        // vector's first component whatever the index
        const f32x4 af = __builtin_bit_cast(f32x4, a);
        const f32x4 bf = __builtin_bit_cast(f32x4, b);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af.x, bf.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af.y, bf.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af.z, bf.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af.w, bf.w, acc, 0, 0, 0);
    }
    static __device__ __forceinline__ Frag load_g(Rsrc r, int voff, int soff) { return buf_load16(r, voff, soff); }
    static __device__ __forceinline__ Frag load_s(const char *p) { return *(const u32x4 *)p; }
};

template <>
struct Mma<kBF16> {
    using Frag = u32x4;
    static __device__ __forceinline__ void run(f32x16 &acc, const Frag &a, const Frag &b, int)
    {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                      __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    static __device__ __forceinline__ Frag load_g(Rsrc r, int voff, int soff) { return buf_load16(r, voff, soff); }
    static __device__ __forceinline__ Frag load_s(const char *p) { return *(const u32x4 *)p; }
};

template <>
struct Mma<kFP8> {
    using Frag = i32x8;
    // acc += 2^(sc - 127) (a . b): format 0 = OCP e4m3 for both operands; the E8M0 scale sc
    // of the weight operand carries the layer's power-of-two factor (the activation operand's
    // scale is 127 = 2^0).  Scaling by a power of two is exact, so this equals scaling the
    // plain sum.
    static __device__ __forceinline__ void run(f32x16 &acc, const Frag &a, const Frag &b, int sc)
    {
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, sc, 0, 127);
    }
    static __device__ __forceinline__ Frag cat(u32x4 lo, u32x4 hi)
    {
        return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                     (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    static __device__ __forceinline__ Frag load_g(Rsrc r, int voff, int soff)
    {
        return cat(buf_load16(r, voff, soff), buf_load16(r, voff + 16, soff));
    }
    static __device__ __forceinline__ Frag load_s(const char *p)
    {
        return cat(*(const u32x4 *)p, *(const u32x4 *)(p + 16));
    }
};

template <int... Is, typename F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, F &&f)
{
    (f(std::integral_constant<int, Is>{}), ...);
}

// Calls f(integral_constant<int, i>) for i = 0 .. N-1: every index is a compile-time constant,
// so register arrays indexed by it stay in registers.
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

// acc[r][c] += W[T0 + r] (k-blocks 0..NKB-1) x act[column tile col0 + c] for one wave, k-block
// loop fully unrolled; hook(kb) runs after the MFMAs of k-block kb are issued (used to
// overlap the previous pass's epilogue with this pass's matrix work).
// Weight fragment (T, kb) of lane l lives at wA + ((T * NKB + kb) * 64 + l) * frag_bytes: one
// contiguous 1 KB (2 KB for FP8) line per wave.  B operand of lane (n, h) for column tile c and
// k-block kb: LDS row 32 c + n, bytes [kb * KBB + h * KBB / 2, ... + KBB / 2).
// A fragments are prefetched two k-blocks ahead, B fragments one.
template <int P, int RP, int CT, int NKB, typename Hook>
__device__ __forceinline__ void mma_pass(f32x16 (&acc)[RP][CT], Rsrc wA, int T0, const char *act,
                                         int stride, int col0, int lane, Hook &&hook, int sc = 127)
{
    using M = Mma<P>;
    using Frag = typename M::Frag;
    constexpr int FB = frag_bytes(P);
    constexpr int KBB = kb_width(P) * elem_bytes(P);
    const int h = lane >> 5, n = lane & 31;
    const int t0 = __builtin_amdgcn_readfirstlane(T0);     // wave-uniform: scalar offsets
    const int voff = lane * FB;
    const char *sb = act + (col0 * 32 + n) * stride + h * (KBB / 2);
    Frag a[3][RP], b[2][CT];
    auto loadA = [&](int slot, int kb) {
#pragma unroll
        for (int r = 0; r < RP; ++r) a[slot][r] = M::load_g(wA, voff, ((t0 + r) * NKB + kb) * 64 * FB);
    };
    auto loadB = [&](int slot, int kb) {
#pragma unroll
        for (int c = 0; c < CT; ++c) b[slot][c] = M::load_s(sb + c * 32 * stride + kb * KBB);
    };
    loadA(0, 0);
    if constexpr (NKB > 1) loadA(1, 1);
    loadB(0, 0);
    sfor<NKB>([&](auto KB) {
        constexpr int kb = decltype(KB)::value;
        if constexpr (kb + 2 < NKB) loadA((kb + 2) % 3, kb + 2);
        if constexpr (kb + 1 < NKB) loadB((kb + 1) % 2, kb + 1);
#pragma unroll
        for (int r = 0; r < RP; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) M::run(acc[r][c], a[kb % 3][r], b[kb % 2][c], sc);
        hook(KB);
        // keep each k-block in its own scheduling region: otherwise the scheduler merges the
        // passes' k-loops (they are independent), which defeats both the prefetch distance and
        // the epilogue overlap and raises register pressure
        __builtin_amdgcn_sched_barrier(0);
    });
}

// acc[r][c][i] = bias of output row 32 * (T0 + r) + 8 * (i / 4) + 4 * h + i % 4.
template <int RP, int CT>
__device__ __forceinline__ void init_bias(f32x16 (&acc)[RP][CT], Rsrc bias, int T0, int lane)
{
    const int h = lane >> 5;
    const int t0 = __builtin_amdgcn_readfirstlane(T0);
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        f32x16 v;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const f32x4 b4 = __builtin_bit_cast(f32x4, buf_load16(bias, (8 * g + 4 * h) * 4, 32 * (t0 + r) * 4));
            v[4 * g + 0] = b4.x;
            v[4 * g + 1] = b4.y;
            v[4 * g + 2] = b4.z;
            v[4 * g + 3] = b4.w;
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[r][c] = v;
    }
}

__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

__device__ __forceinline__ uint32_t pack_fp8x4(float a, float b, float c, float d)
{
    // saturate to the largest finite e4m3 value (one median-of-three each)
    a = __builtin_amdgcn_fmed3f(a, -448.0f, 448.0f);
    b = __builtin_amdgcn_fmed3f(b, -448.0f, 448.0f);
    c = __builtin_amdgcn_fmed3f(c, -448.0f, 448.0f);
    d = __builtin_amdgcn_fmed3f(d, -448.0f, 448.0f);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

// 32-bit words one epilogue unit (4 consecutive accumulator values) packs into.
__host__ __device__ constexpr int words_per_unit(int po) { return po == kF32 ? 4 : (po == kBF16 ? 2 : 1); }

// Store the packed epilogue of accumulator tile (row tile T, column tile c) into the LDS
// activation tile in the column order that a consumer with operand precision PO reads
// (see phys_to_feature()).
template <int PO>
__device__ __forceinline__ void store_tile(const uint32_t *w, int T, int c, char *act, int stride,
                                           int lane)
{
    const int h = lane >> 5, n = lane & 31;
    char *row = act + (c * 32 + n) * stride;
    if constexpr (PO == kF32) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
            *(u32x4 *)(row + ((4 * T + g) * 8 + 4 * h) * 4) =
                u32x4{w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3]};
    } else if constexpr (PO == kBF16) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
            *(u32x4 *)(row + ((2 * T + q) * 16 + 8 * h) * 2) =
                u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
    } else {
        *(u32x4 *)(row + (T / 2) * 64 + 32 * h + 16 * (T % 2)) = u32x4{w[0], w[1], w[2], w[3]};
    }
}

// k-block visiting orders.  The activation tile's k-blocks split into two halves: those holding
// the outputs of the producing layer's first row pass ("half 0") and those of its second
// ("half 1"); G consecutive k-blocks belong to one pass of one wave.
struct MapAll {
    static constexpr int kb(int j) { return j; }
};
template <int G>
struct MapHalf0 {
    static constexpr int kb(int j) { return (j / G) * 2 * G + j % G; }
};
template <int G>
struct MapHalf1 {
    static constexpr int kb(int j) { return (j / G) * 2 * G + G + j % G; }
};

// acc[r][c] += W[T0 + r] x act[column tile col0 + c] over the NJ k-blocks Map::kb(0..NJ-1) of
// a layer with NKB k-blocks (same fragment layout and prefetch scheme as mma_pass).
template <int P, int RP, int CT, int NKB, int NJ, typename Map, int VPM = 0, int SWAPB = 0, typename Hook>
__device__ __forceinline__ void mma_seq(f32x16 (&acc)[RP][CT], Rsrc wA, int T0, const char *act,
                                        int stride, int col0, int lane, Hook &&hook, int sc = 127)
{
    constexpr int MFMA_PER_RUN = (P == kF32) ? 4 : 1;
    using M = Mma<P>;
    using Frag = typename M::Frag;
    constexpr int FB = frag_bytes(P);
    constexpr int KBB = kb_width(P) * elem_bytes(P);
    const int h = lane >> 5, n = lane & 31;
    const int t0 = __builtin_amdgcn_readfirstlane(T0);
    const int voff = lane * FB;
    const char *sb = act + (col0 * 32 + n) * stride + h * (KBB / 2);
    // k-blocks the weight loads run ahead (an FP8 k-block is four times the matrix work of a
    // BF16 one, and its fragments twice the registers)
    constexpr int PA = (P == kFP8) ? 1 : GMC_PFA;
    Frag a[PA + 1][RP], b[2][CT];
    auto loadA = [&](int slot, int kb) {
#pragma unroll
        for (int r = 0; r < RP; ++r) a[slot][r] = M::load_g(wA, voff, ((t0 + r) * NKB + kb) * 64 * FB);
    };
    auto loadB = [&](int slot, int kb) {
#pragma unroll
        for (int c = 0; c < CT; ++c) b[slot][c] = M::load_s(sb + c * 32 * stride + (kb ^ SWAPB) * KBB);
    };
    sfor<PA>([&](auto I) {
        if constexpr (decltype(I)::value < NJ) loadA(decltype(I)::value, Map::kb(decltype(I)::value));
    });
    loadB(0, Map::kb(0));
    sfor<NJ>([&](auto JJ) {
        constexpr int j = decltype(JJ)::value;
        if constexpr (j + PA < NJ) loadA((j + PA) % (PA + 1), Map::kb(j + PA));
        if constexpr (j + 1 < NJ) loadB((j + 1) % 2, Map::kb(j + 1));
#pragma unroll
        for (int r = 0; r < RP; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) M::run(acc[r][c], a[j % (PA + 1)][r], b[j % 2][c], sc);
        hook(JJ);
        if constexpr (VPM > 0) {
            // interleave the hook's epilogue arithmetic between the MFMAs: one MFMA, then up
            // to VPM vector instructions, so transcendental latencies hide behind matrix work
            sfor<RP * CT * MFMA_PER_RUN>([&](auto) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, VPM, 0);
            });
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Noise z and condition features cf of sample i of a launch (paper "Transport Algorithm",
// second stage: noise drawn from the sample's Philox stream unless given).  Condition features:
// boundary model (ln tau, c, 2 y_in - 1, sin th, f4, 0) with f4 = ln A for rectangular cells,
// the entry direction's in-plane x component omega_x for an XY-geometry model, else 0; internal
// model (ln tau, c, 2 x - 1, 2 y - 1, cos phi, sin phi).  Indices past n_items get zero noise
// and a neutral condition (their results are not stored).
__device__ __forceinline__ void sampler_inputs(const MlpParams &p, int64_t i, int64_t n_items, float z[5],
                                               float cf[6])
{
    float lt = 0.f, cc = 0.f, yy = 0.5f, ss = 0.f, xx = 0.5f, co = 1.f, la = 0.f;
#pragma unroll
    for (int d = 0; d < 5; ++d) z[d] = 0.0f;
    if (i < n_items) {
        lt = p.log_tau[i];
        cc = p.c[i];
        yy = p.y_in[i];
        ss = p.sin_th[i];
        if (p.n_cond == 6) {
            xx = p.x_in[i];
            co = p.cos_phi[i];
        }
        if (p.log_aspect) la = p.log_aspect[i];
        else if (p.omega_x) la = p.omega_x[i];
        if (p.noise) {
#pragma unroll
            for (int d = 0; d < 5; ++d) z[d] = p.noise[d * p.n + i];
        } else {
            normal5(p.keys ? p.keys[i] : p.seed, p.ids ? p.ids[i] : p.id_base + (uint64_t)i, z);
        }
    }
    cf[0] = lt;
    cf[1] = cc;
    if (p.n_cond == 6) {
        cf[2] = 2.0f * xx - 1.0f;
        cf[3] = 2.0f * yy - 1.0f;
        cf[4] = co;
        cf[5] = ss;
    } else {
        cf[2] = 2.0f * yy - 1.0f;
        cf[3] = ss;
        cf[4] = la;
        cf[5] = 0.0f;
    }
}

// Stores sample i's final state: the raw network state (if asked for) and the decoded exit
// record (eq. 11).
__device__ __forceinline__ void sampler_outputs(const MlpParams &p, int64_t i, const float xk[5])
{
    if (p.raw) {
#pragma unroll
        for (int d = 0; d < 5; ++d) p.raw[d * p.n + i] = xk[d];
    }
    Exit e;
    decode_exit(xk[0], xk[1], xk[2], xk[3], xk[4], e, p.xy != 0);
    p.face[i] = e.face;
    p.pos[i] = e.pos;
    p.dcos[i] = e.u;
    p.dsin[i] = e.v;
    p.path[i] = e.path;
}

}  // namespace
}  // namespace gmc
