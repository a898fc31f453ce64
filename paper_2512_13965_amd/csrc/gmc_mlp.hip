// Fused velocity-MLP + Euler ODE sampler for gfx950 (paper: section "Conditional Flow
// Matching", eq. 8; network of section "Network Architecture and Inputs"; decoding of eq. 11).
//
// One persistent workgroup per CU (4 waves, 256 lanes) owns a tile of 128 samples at a time and
// carries it through all K Euler steps x <- x + v(x, k/K | c) / K:
//   * the tile's activations live in LDS (128 x H), the ODE state x and the condition in LDS;
//   * each hidden layer is a [H x H] x [H x 128] contraction on MFMA; wave w owns the output
//     rows [w*H/4, (w+1)*H/4) and keeps its 32x32 accumulator tiles in registers;
//   * weights stream from L2 straight into MFMA operand registers, pre-arranged on the host in
//     per-lane fragment order so each lane issues one 16-byte load per 32-row tile and k-block
//     and a wave's loads are one contiguous 1 KB line;
//   * the epilogue (bias already in the accumulator, SiLU, cast to the next layer's operand
//     type) writes each accumulator tile back into the LDS activation tile in the column order
//     the next layer's operand reads expect, so the next layer's B-operand reads are contiguous
//     16-byte LDS reads; the host permutes the next layer's weight columns to match.
#include "gmc_device.hpp"
#include "gmc_internal.hpp"

namespace gmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int P>
struct Mma;

template <>
struct Mma<kF32> {
    using Frag = u32x4;
    static __device__ __forceinline__ void run(f32x16 &acc, const Frag &a, const Frag &b)
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
    static __device__ __forceinline__ Frag load_g(const char *p) { return *(const u32x4 *)p; }
    static __device__ __forceinline__ Frag load_s(const char *p) { return *(const u32x4 *)p; }
};

template <>
struct Mma<kBF16> {
    using Frag = u32x4;
    static __device__ __forceinline__ void run(f32x16 &acc, const Frag &a, const Frag &b)
    {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                      __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    static __device__ __forceinline__ Frag load_g(const char *p) { return *(const u32x4 *)p; }
    static __device__ __forceinline__ Frag load_s(const char *p) { return *(const u32x4 *)p; }
};

template <>
struct Mma<kFP8> {
    using Frag = i32x8;
    static __device__ __forceinline__ void run(f32x16 &acc, const Frag &a, const Frag &b)
    {
        // format 0 = OCP e4m3 for both operands; E8M0 scales of 127 = 2^0 (scaling is done in
        // the epilogue with the per-layer power-of-two factors)
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
    }
    static __device__ __forceinline__ Frag load_g(const char *p)
    {
        const u32x4 lo = *(const u32x4 *)p, hi = *(const u32x4 *)(p + 16);
        return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                     (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    static __device__ __forceinline__ Frag load_s(const char *p) { return load_g(p); }
};

// acc[r][c] += W[tile0 + r] (k-blocks 0..NKB-1) x act[col tile c] for one wave.
// Weight fragment (T, kb) of lane l lives at wA + ((T * NKB + kb) * 64 + l) * frag_bytes.
// B operand of lane (n, h) for column tile c and k-block kb: LDS row 32c + n, columns
// kb * W + h * W / 2 ... + W / 2 - 1 (W = k-block width), one contiguous chunk.
template <int P, int RT, int CT, int NKB>
__device__ __forceinline__ void mma_layer(f32x16 (&acc)[RT][CT], const char *__restrict__ wA,
                                          int tile0, const char *act, int stride, int col0,
                                          int lane)
{
    using M = Mma<P>;
    using Frag = typename M::Frag;
    constexpr int FB = frag_bytes(P);
    constexpr int KBB = kb_width(P) * elem_bytes(P);   // bytes of one k-block in an LDS row
    const int h = lane >> 5, n = lane & 31;
    const char *ga = wA + ((size_t)tile0 * NKB * 64 + lane) * FB;
    const char *sb = act + (col0 * 32 + n) * stride + h * (KBB / 2);
    Frag a[2][RT], b[2][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r) a[0][r] = M::load_g(ga + (size_t)r * NKB * 64 * FB);
#pragma unroll
    for (int c = 0; c < CT; ++c) b[0][c] = M::load_s(sb + c * 32 * stride);
#pragma unroll 2
    for (int kb = 0; kb < NKB; ++kb) {
        const int cur = kb & 1, nxt = cur ^ 1;
        if (kb + 1 < NKB) {
#pragma unroll
            for (int r = 0; r < RT; ++r)
                a[nxt][r] = M::load_g(ga + ((size_t)r * NKB + kb + 1) * 64 * FB);
#pragma unroll
            for (int c = 0; c < CT; ++c) b[nxt][c] = M::load_s(sb + c * 32 * stride + (kb + 1) * KBB);
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) M::run(acc[r][c], a[cur][r], b[cur][c]);
    }
}

// acc[r][c][i] = bias of output row 32 * (tile0 + r) + 8 * (i / 4) + 4 * h + i % 4.
template <int RT, int CT>
__device__ __forceinline__ void init_bias(f32x16 (&acc)[RT][CT], const float *__restrict__ bias,
                                          int tile0, int lane)
{
    const int h = lane >> 5;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        f32x16 v;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const f32x4 b4 = *(const f32x4 *)(bias + 32 * (tile0 + r) + 8 * g + 4 * h);
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
    a = fminf(fmaxf(a, -448.0f), 448.0f);
    b = fminf(fmaxf(b, -448.0f), 448.0f);
    c = fminf(fmaxf(c, -448.0f), 448.0f);
    d = fminf(fmaxf(d, -448.0f), 448.0f);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

// SiLU(acc * oscale) * inv_next written into the LDS activation tile in the column order of a
// consumer with operand precision PO (see phys_to_feature()).
template <int PO, int RT, int CT>
__device__ __forceinline__ void epilogue(const f32x16 (&acc)[RT][CT], int tile0, char *act,
                                         int stride, int lane, float oscale, float inv_next)
{
    const int h = lane >> 5, n = lane & 31;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int T = tile0 + r;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            char *row = act + (c * 32 + n) * stride;
            float y[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) y[i] = silu(acc[r][c][i] * oscale) * inv_next;
            if constexpr (PO == kF32) {
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    *(f32x4 *)(row + ((4 * T + g) * 8 + 4 * h) * 4) =
                        f32x4{y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
            } else if constexpr (PO == kBF16) {
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    *(u32x4 *)(row + ((2 * T + q) * 16 + 8 * h) * 2) =
                        u32x4{pack_bf16(y[8 * q], y[8 * q + 1]), pack_bf16(y[8 * q + 2], y[8 * q + 3]),
                              pack_bf16(y[8 * q + 4], y[8 * q + 5]), pack_bf16(y[8 * q + 6], y[8 * q + 7])};
            } else {
                *(u32x4 *)(row + (T / 2) * 64 + 32 * h + 16 * (T % 2)) =
                    u32x4{pack_fp8x4(y[0], y[1], y[2], y[3]), pack_fp8x4(y[4], y[5], y[6], y[7]),
                          pack_fp8x4(y[8], y[9], y[10], y[11]), pack_fp8x4(y[12], y[13], y[14], y[15])};
            }
        }
    }
}

template <int MP, int H>
struct Cfg {
    static constexpr int P1 = layer_prec(MP, 0);            // layer 1 operand precision
    static constexpr int PH = layer_prec(MP, 1);            // hidden layers' operand precision
    static constexpr int P5 = layer_prec(MP, 4);            // last layer operand precision
    static constexpr int ACT_ELEM = (MP == kF32) ? 4 : 2;   // widest type stored in the tile
    static constexpr int ACT_STRIDE = H * ACT_ELEM + 16;    // +16 B: conflict-free row reads
    static constexpr int IN_STRIDE = 16 * elem_bytes(P1) + 16;
    static constexpr int RT = H / (32 * kWaves);            // row tiles per wave
    static constexpr int NKB1 = 16 / kb_width(P1);
    static constexpr int NKBH = H / kb_width(PH);
    static constexpr int NKB5 = H / kb_width(P5);
    static constexpr int LDS_ACT = kTileM * ACT_STRIDE;
    static constexpr int LDS_IN = kTileM * IN_STRIDE;
    static constexpr int LDS_BYTES = LDS_ACT + LDS_IN + (5 + 4) * kTileM * 4;
};

template <int MP, int H>
__global__ __launch_bounds__(256, 1) void mlp_ode_kernel(MlpParams p)
{
    using C = Cfg<MP, H>;
    static_assert(C::LDS_BYTES <= 160 * 1024, "LDS budget");
    __shared__ __attribute__((aligned(16))) char smem[C::LDS_BYTES];
    char *act = smem;
    char *in0 = smem + C::LDS_ACT;
    float *xs = (float *)(smem + C::LDS_ACT + C::LDS_IN);   // [5][128] ODE state
    float *cf = xs + 5 * kTileM;                              // [4][128] condition features

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t ntiles = (p.n + kTileM - 1) / kTileM;
    const float dt = 1.0f / (float)p.K;
    const int tile0 = wave * C::RT;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * kTileM;
        if (tid < kTileM) {
            const int64_t i = base + tid;
            float z[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            float lt = 0.f, cc = 0.f, yy = 0.5f, ss = 0.f;
            if (i < p.n) {
                lt = p.log_tau[i];
                cc = p.c[i];
                yy = p.y_in[i];
                ss = p.sin_th[i];
                if (p.noise) {
#pragma unroll
                    for (int d = 0; d < 5; ++d) z[d] = p.noise[d * p.n + i];
                } else {
                    normal5(p.seed, p.id_base + (uint64_t)i, z);
                }
            }
#pragma unroll
            for (int d = 0; d < 5; ++d) xs[d * kTileM + tid] = z[d];
            cf[0 * kTileM + tid] = lt;
            cf[1 * kTileM + tid] = cc;
            cf[2 * kTileM + tid] = 2.0f * yy - 1.0f;
            cf[3 * kTileM + tid] = ss;
        }
        __syncthreads();

        for (int k = 0; k < p.K; ++k) {
            const float t = (float)k * dt;
            // layer-1 input row of sample sn: [x0..x4, t, ln tau, c, 2y-1, sin th, 0 x 6]
            {
                const int sn = tid & (kTileM - 1), half = tid >> 7;
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int q = 8 * half + j;
                    v[j] = q < 5 ? xs[q * kTileM + sn]
                                 : (q == 5 ? t : (q < 10 ? cf[(q - 6) * kTileM + sn] : 0.0f));
                }
                char *row = in0 + sn * C::IN_STRIDE;
                if constexpr (C::P1 == kF32) {
                    *(f32x4 *)(row + 32 * half) = f32x4{v[0], v[1], v[2], v[3]};
                    *(f32x4 *)(row + 32 * half + 16) = f32x4{v[4], v[5], v[6], v[7]};
                } else {
                    *(u32x4 *)(row + 16 * half) = u32x4{pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]),
                                                        pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7])};
                }
            }
            __syncthreads();

            f32x16 acc[C::RT][4];
            // layer 1: 10 -> H
            init_bias<C::RT, 4>(acc, p.bias[0], tile0, lane);
            mma_layer<C::P1, C::RT, 4, C::NKB1>(acc, (const char *)p.wA[0], tile0, in0, C::IN_STRIDE, 0, lane);
            epilogue<C::PH, C::RT, 4>(acc, tile0, act, C::ACT_STRIDE, lane, p.oscale[0], p.inv_in_scale[1]);
            __syncthreads();
            // hidden layers 2..4: H -> H
#pragma unroll 1
            for (int l = 1; l < 4; ++l) {
                init_bias<C::RT, 4>(acc, p.bias[l], tile0, lane);
                mma_layer<C::PH, C::RT, 4, C::NKBH>(acc, (const char *)p.wA[l], tile0, act, C::ACT_STRIDE, 0, lane);
                __syncthreads();
                if (l < 3)
                    epilogue<C::PH, C::RT, 4>(acc, tile0, act, C::ACT_STRIDE, lane, p.oscale[l], p.inv_in_scale[l + 1]);
                else
                    epilogue<C::P5, C::RT, 4>(acc, tile0, act, C::ACT_STRIDE, lane, p.oscale[l], 1.0f);
                __syncthreads();
            }
            // layer 5: H -> 5 (rows padded to 32); wave w handles sample column tile w
            {
                f32x16 out[1][1];
                init_bias<1, 1>(out, p.bias[4], 0, lane);
                mma_layer<C::P5, 1, 1, C::NKB5>(out, (const char *)p.wA[4], 0, act, C::ACT_STRIDE, wave, lane);
                const int sn = wave * 32 + (lane & 31);
                if (lane < 32) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) xs[d * kTileM + sn] += out[0][0][d] * dt;
                } else {
                    xs[4 * kTileM + sn] += out[0][0][0] * dt;
                }
            }
            __syncthreads();
        }

        if (tid < kTileM) {
            const int64_t i = base + tid;
            if (i < p.n) {
                const float a0 = xs[0 * kTileM + tid], a1 = xs[1 * kTileM + tid],
                            a2 = xs[2 * kTileM + tid], a3 = xs[3 * kTileM + tid],
                            a4 = xs[4 * kTileM + tid];
                if (p.raw) {
                    p.raw[0 * p.n + i] = a0;
                    p.raw[1 * p.n + i] = a1;
                    p.raw[2 * p.n + i] = a2;
                    p.raw[3 * p.n + i] = a3;
                    p.raw[4 * p.n + i] = a4;
                }
                Exit e;
                decode_exit(a0, a1, a2, a3, a4, e);
                p.face[i] = e.face;
                p.pos[i] = e.pos;
                p.dcos[i] = e.u;
                p.dsin[i] = e.v;
                p.path[i] = e.path;
            }
        }
        __syncthreads();
    }
}

template <int MP, int H>
hipError_t launch_one(const MlpParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((mlp_ode_kernel<MP, H>), dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace

bool mlp_supported(int prec, int hidden)
{
    if (prec == kF32) return hidden == 128 || hidden == 256;
    if (prec == kBF16 || prec == kFP8) return hidden == 128 || hidden == 256 || hidden == 512;
    return false;
}

hipError_t launch_mlp_ode(int prec, int hidden, const MlpParams &p, int grid, hipStream_t s)
{
    switch (prec * 1000 + hidden) {
    case kF32 * 1000 + 128: return launch_one<kF32, 128>(p, grid, s);
    case kF32 * 1000 + 256: return launch_one<kF32, 256>(p, grid, s);
    case kBF16 * 1000 + 128: return launch_one<kBF16, 128>(p, grid, s);
    case kBF16 * 1000 + 256: return launch_one<kBF16, 256>(p, grid, s);
    case kBF16 * 1000 + 512: return launch_one<kBF16, 512>(p, grid, s);
    case kFP8 * 1000 + 128: return launch_one<kFP8, 128>(p, grid, s);
    case kFP8 * 1000 + 256: return launch_one<kFP8, 256>(p, grid, s);
    case kFP8 * 1000 + 512: return launch_one<kFP8, 512>(p, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gmc
