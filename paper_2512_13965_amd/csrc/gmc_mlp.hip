// Fused velocity-MLP + ODE sampler for gfx950 (paper: section "Conditional Flow
// Matching", eq. 8; network of section "Network Architecture and Inputs"; decoding of eq. 11).
//
// Persistent workgroups (four waves, or eight in the two-group schedule of BF16 / FP8 models
// of width 256 and more) each own a tile of samples at a time and carry it through all ODE
// steps (Euler x <- x + v(x, k/K | c) / K, or classic RK4):
//   * the tile's activations live in LDS (128 x H), the ODE state x and the condition in LDS;
//   * each hidden layer is a [H x H] x [H x 128] contraction on MFMA; each wave owns a set of
//     32-row output tiles (four-wave kernels: wave w the rows [w*H/4, (w+1)*H/4); two-group
//     schedule: see Cfg) and keeps its 32x32 accumulator tiles in registers;
//   * weights stream from L2 straight into MFMA operand registers, pre-arranged on the host in
//     per-lane fragment order so each lane issues one 16-byte load per 32-row tile and k-block
//     and a wave's loads are one contiguous 1 KB line;
//   * the epilogue (bias already in the accumulator, SiLU, cast to the next layer's operand
//     type) writes each accumulator tile back into the LDS activation tile in the column order
//     the next layer's operand reads expect, so the next layer's B-operand reads are contiguous
//     16-byte LDS reads; the host permutes the next layer's weight columns to match.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "gmc_device.hpp"
#include "gmc_internal.hpp"
#include "gmc_mma.hpp"

// MFMA / epilogue interleave: vector instructions placed after each MFMA in the overlapped
// k-loops (0 = leave the order to the scheduler).
#ifndef GMC_VPM_A
#define GMC_VPM_A 0
#endif
#ifndef GMC_VPM_P
#define GMC_VPM_P 0
#endif
#ifndef GMC_VPM_5
#define GMC_VPM_5 0
#endif
#ifndef GMC_DRAIN_STAGED
#define GMC_DRAIN_STAGED 1
#endif
#ifndef GMC_DRAIN_W
#define GMC_DRAIN_W 16
#endif
// Drains of the two-group schedule: 1 = software-pipelined epilogue (drain_pipe), 0 = one
// accumulator tile at a time (epi_tile).  GMC_PIPE_D: iterations between a value's stages.
#ifndef GMC_DRAIN_PIPE
#define GMC_DRAIN_PIPE 1
#endif
#ifndef GMC_PIPE_D
#define GMC_PIPE_D 1
#endif
// 8: BF16 / FP8 models of width >= 256 use the two-group schedule (eight waves); 4: they use
// the single-group cross-layer pipeline (four waves).  Both give bit-identical results.
#ifndef GMC_WIDE_WAVES
#define GMC_WIDE_WAVES 8
#endif
// Largest number of persistent workgroups per compute unit for the four-wave kernels (FP32, and
// BF16 / FP8 at width 128), as far as registers and LDS allow.
#ifndef GMC_MAX_WG_PER_CU
#define GMC_MAX_WG_PER_CU 4
#endif

namespace gmc {
namespace {

// BF16 and FP8 models carry every hidden activation scaled by -log2(e): the host scales the
// first layer's weights and every hidden bias by -log2(e) and the output layer's weights by
// -ln 2 (the same network in exact arithmetic), so an accumulator holds a' = -log2(e) a, and
// the scaled activation -log2(e) SiLU(a) is a' / (1 + 2^a'): the exponential takes the
// accumulator as it is.  FP8 models (SCALE) store half of it divided by the next layer's
// activation scale (a power of two, folded into the reciprocal's argument) and their e4m3
// layers apply 2 sw sa through the matrix core's operand scale.  FP32 models keep plain
// activations.
template <int PO, bool SCALE>
constexpr bool exp2_folded()
{
    return SCALE || PO == kBF16;
}

// -log2(e) SiLU(a) from a' = -log2(e) a.
__device__ __forceinline__ float silu_exp2(float a)
{
    return a * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a));
}

// Multiplier of the accumulator that gives the exponential's argument: -log2(e) times the
// scaled pre-activation, or 1 where the activations carry that factor already.
template <int PO, bool SCALE>
__device__ __forceinline__ float exp2_factor(float)
{
    if constexpr (exp2_folded<PO, SCALE>()) return 1.0f;
    else return -1.4426950408889634f;
}

// One epilogue unit: the activation of accumulator values 4g .. 4g+3 times oscale * inv_next,
// packed in the consumer's operand type (BF16 and FP8 models: the scaled activation, see
// exp2_folded).
template <int PO, bool SCALE>
__device__ __forceinline__ void epi_unit(const f32x16 &acc, int g, float oscale, float inv_next,
                                         uint32_t *w)
{
    float y[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float a = acc[4 * g + j];
        if constexpr (SCALE) y[j] = silu_exp2(a) * (oscale * inv_next);
        else if constexpr (exp2_folded<PO, SCALE>()) y[j] = silu_exp2(a);
        else y[j] = silu(a);
    }
    if constexpr (PO == kF32) {
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = __builtin_bit_cast(uint32_t, y[j]);
    } else if constexpr (PO == kBF16) {
        w[0] = pack_bf16(y[0], y[1]);
        w[1] = pack_bf16(y[2], y[3]);
    } else {
        w[0] = pack_fp8x4(y[0], y[1], y[2], y[3]);
    }
}

// The epilogue of a whole accumulator tile (16 values per lane): the operations of epi_unit,
// issued stage by stage over DW values so that independent transcendentals follow each other.
template <int PO, bool SCALE>
__device__ __forceinline__ void epi_tile(const f32x16 &acc, float oscale, float inv_next, uint32_t *w)
{
#if GMC_DRAIN_STAGED
    constexpr int DW = GMC_DRAIN_W;
    // acc * c1 is the exponential's argument (c1 = 1 where the accumulator carries -log2(e));
    // with per-layer scales (powers of two) (acc * c2) * sigmoid is (acc * sigmoid) * c2 with
    // its single rounding, since scaling by a power of two is exact.
    const float c1 = exp2_factor<PO, SCALE>(oscale);
    const float c2 = oscale * inv_next;
    sfor<16 / DW>([&](auto HH) {
        constexpr int h0 = decltype(HH)::value * DW;
        float a[DW], t[DW];
#pragma unroll
        for (int i = 0; i < DW; ++i) {
            a[i] = SCALE ? acc[h0 + i] * c2 : acc[h0 + i];
            t[i] = c1 * acc[h0 + i];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < DW; ++i) t[i] = __builtin_amdgcn_exp2f(t[i]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < DW; ++i) t[i] = __builtin_amdgcn_rcpf(1.0f + t[i]);
        __builtin_amdgcn_sched_barrier(0);
        float y[DW];
#pragma unroll
        for (int i = 0; i < DW; ++i) y[i] = a[i] * t[i];
        if constexpr (PO == kF32) {
#pragma unroll
            for (int i = 0; i < DW; ++i) w[h0 + i] = __builtin_bit_cast(uint32_t, y[i]);
        } else if constexpr (PO == kBF16) {
#pragma unroll
            for (int i = 0; i < DW / 2; ++i) w[h0 / 2 + i] = pack_bf16(y[2 * i], y[2 * i + 1]);
        } else {
#pragma unroll
            for (int i = 0; i < DW / 4; ++i) w[h0 / 4 + i] = pack_fp8x4(y[4 * i], y[4 * i + 1], y[4 * i + 2], y[4 * i + 3]);
        }
    });
#else
    constexpr int WPU = words_per_unit(PO);
#pragma unroll
    for (int g = 0; g < 4; ++g) epi_unit<PO, SCALE>(acc, g, oscale, inv_next, &w[g * WPU]);
#endif
}

// The SiLU epilogue of the NT accumulator tiles a(t) (16 values each, value i = 16 t + i % 16),
// software-pipelined: iteration j issues the first multiply of value j, the exponential of value
// j - D, the add of value j - 2D, the reciprocal of value j - 3D and the final multiply of value
// j - 4D -- independent instructions -- and packs groups of values as they complete;
// store(t, words) receives each tile's packed words (the layout of epi_tile) once its last value
// is done.  The arithmetic is epi_tile's: acc * c1 is -log2(e) times the pre-activation (c1 = 1
// in BF16 and FP8 models, whose accumulators carry the factor: the multiply drops out), and
// with per-layer scales the output factor c2 = oscale * inv_next (a power of two) moves into
// the reciprocal's argument, acc * rcp((1 + e) / c2) being exactly (acc * c2) * rcp(1 + e).
template <int PO, bool SCALE, int NT, typename Val, typename Store>
__device__ __forceinline__ void drain_pipe(Val &&val, float oscale, float inv_next, Store &&store)
{
    constexpr int NV = NT * 16;
    constexpr int D = GMC_PIPE_D;
    const float c1 = exp2_factor<PO, SCALE>(oscale);
    const float k = SCALE ? 1.0f / (oscale * inv_next) : 1.0f;
    float t[NV], y[NV];
    uint32_t wd[NT][4 * words_per_unit(PO)];
    sfor<NV + 4 * D>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if constexpr (j < NV) t[j] = c1 * val(std::integral_constant<int, j>{});
        if constexpr (j - D >= 0 && j - D < NV) t[j - D] = __builtin_amdgcn_exp2f(t[j - D]);
        if constexpr (j - 2 * D >= 0 && j - 2 * D < NV) {
            if constexpr (SCALE) t[j - 2 * D] = __builtin_fmaf(t[j - 2 * D], k, k);
            else t[j - 2 * D] = 1.0f + t[j - 2 * D];
        }
        if constexpr (j - 3 * D >= 0 && j - 3 * D < NV) t[j - 3 * D] = __builtin_amdgcn_rcpf(t[j - 3 * D]);
        if constexpr (j - 4 * D >= 0 && j - 4 * D < NV) {
            constexpr int i = j - 4 * D;
            y[i] = val(std::integral_constant<int, i>{}) * t[i];
            constexpr int tt = i / 16, v = i % 16;
            if constexpr (PO == kF32) {
                wd[tt][v] = __builtin_bit_cast(uint32_t, y[i]);
            } else if constexpr (PO == kBF16) {
                if constexpr (v % 2 == 1) wd[tt][v / 2] = pack_bf16(y[i - 1], y[i]);
            } else {
                if constexpr (v % 4 == 3) wd[tt][v / 4] = pack_fp8x4(y[i - 3], y[i - 2], y[i - 1], y[i]);
            }
            if constexpr (v == 15) store(std::integral_constant<int, tt>{}, wd[tt]);
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}


// One dense layer + SiLU for this wave's RTW row tiles and all 128 samples of the tile.  The
// rows are done in NP passes of RP row tiles; the epilogue of pass p runs interleaved with the
// MFMA k-loop of pass p + 1 (it only reads pass p's accumulators), so the SiLU transcendentals
// overlap the matrix unit.  Those results are held packed in registers until every wave has
// finished reading the input tile (barrier, when `out` aliases the input); the last pass's
// epilogue is computed and stored after that barrier.
template <int PIN, int POUT, int RTW, int NKB, bool SCALE, bool IN_PLACE>
__device__ __forceinline__ void dense_silu(Rsrc wA, Rsrc bias, int T0, const char *in, int in_stride, char *out,
                                           int out_stride, int lane, float oscale, float inv_next, int sc = 127)
{
    constexpr int RP = RTW >= 4 ? RTW / 2 : 1;     // row tiles per pass
    constexpr int NP = RTW / RP;                   // passes
    constexpr int UNITS = RP * 4 * 4;              // epilogue units (4 values) per pass
    constexpr int WPU = words_per_unit(POUT);
    constexpr int UPK = (UNITS + NKB - 1) / NKB;   // epilogue units per k-block
    uint32_t pk[NP > 1 ? NP - 1 : 1][UNITS * WPU];
    f32x16 acc[2][RP][4];
    auto epi = [&](auto PP, int u) {
        constexpr int pp = decltype(PP)::value;
        const int r = u / 16, c = (u / 4) % 4, g = u % 4;
        epi_unit<POUT, SCALE>(acc[pp % 2][r][c], g, oscale, inv_next, &pk[pp][u * WPU]);
    };
    sfor<NP>([&](auto P) {
        constexpr int p = decltype(P)::value;
        init_bias<RP, 4>(acc[p % 2], bias, T0 + p * RP, lane);
        mma_pass<PIN, RP, 4, NKB>(acc[p % 2], wA, T0 + p * RP, in, in_stride, 0, lane, [&](auto KB) {
            constexpr int kb = decltype(KB)::value;
            if constexpr (p > 0) {
                sfor<UPK>([&](auto J) {
                    constexpr int u = kb * UPK + decltype(J)::value;
                    if constexpr (u < UNITS) epi(std::integral_constant<int, p - 1>{}, u);
                });
            }
        }, sc);
        if constexpr (p > 0 && NKB * UPK < UNITS) {
            sfor<UNITS - NKB * UPK>([&](auto J) {
                epi(std::integral_constant<int, p - 1>{}, NKB * UPK + decltype(J)::value);
            });
        }
    });
    if constexpr (IN_PLACE) __syncthreads();
    sfor<NP - 1>([&](auto P) {
        constexpr int p = decltype(P)::value;
        sfor<RP * 4>([&](auto TC) {
            constexpr int r = decltype(TC)::value / 4, c = decltype(TC)::value % 4;
            store_tile<POUT>(&pk[p][(r * 4 + c) * 4 * WPU], T0 + p * RP + r, c, out, out_stride, lane);
        });
    });
    constexpr int pl = NP - 1;
    sfor<RP * 4>([&](auto TC) {
        constexpr int r = decltype(TC)::value / 4, c = decltype(TC)::value % 4;
        uint32_t w[4 * WPU];
#pragma unroll
        for (int g = 0; g < 4; ++g) epi_unit<POUT, SCALE>(acc[pl % 2][r][c], g, oscale, inv_next, &w[g * WPU]);
        store_tile<POUT>(w, T0 + pl * RP + r, c, out, out_stride, lane);
    });
}

// Part J of NJ of draining accumulator tiles src[RP][4] through the epilogue into packed words.
template <int PO, bool SCALE, int RP, int NJ, int J>
__device__ __forceinline__ void drain_step(const f32x16 (&src)[RP][4], uint32_t *pk, float osc, float inv)
{
    constexpr int UNITS = RP * 16;
    constexpr int UPK = (UNITS + NJ - 1) / NJ;
    constexpr int WPU = words_per_unit(PO);
    sfor<UPK>([&](auto U) {
        constexpr int u = J * UPK + decltype(U)::value;
        if constexpr (u < UNITS) epi_unit<PO, SCALE>(src[u / 16][(u / 4) % 4], u % 4, osc, inv, &pk[u * WPU]);
    });
}

// Store the packed outputs of one row pass (row tiles Tb .. Tb + RP - 1, all column tiles).
template <int PO, int RP>
__device__ __forceinline__ void store_pass(const uint32_t *pk, int Tb, char *act, int stride, int lane)
{
    constexpr int WPU = words_per_unit(PO);
    sfor<RP * 4>([&](auto TC) {
        constexpr int r = decltype(TC)::value / 4, c = decltype(TC)::value % 4;
        store_tile<PO>(&pk[(r * 4 + c) * 4 * WPU], Tb + r, c, act, stride, lane);
    });
}

template <int MP, int H, int TM = kTileM>
struct Cfg {
    static constexpr int P1 = layer_prec(MP, 0);            // layer 1 operand precision
    static constexpr int PH = layer_prec(MP, 1);            // hidden layers' operand precision
    static constexpr int P5 = layer_prec(MP, 4);            // last layer operand precision
    static constexpr bool SCALE = (MP == kFP8);             // per-layer FP8 scales
    static constexpr int ACT_ELEM = (MP == kF32) ? 4 : 2;   // widest type stored in the tile
    static constexpr int ACT_STRIDE = H * ACT_ELEM + 16;    // +16 B: conflict-free row reads
    static constexpr int IN_STRIDE = 16 * elem_bytes(P1) + 16;
    // Two-group schedule (BF16 / FP8, H >= 256): eight waves, two per SIMD.  Group 0 owns the
    // first half of every layer's output rows, group 1 the second half; while one group's
    // waves run the matrix k-loop, the other group's waves run the SiLU epilogue on the same
    // SIMDs, so vector and matrix work overlap across waves.
    static constexpr bool GROUPS = (MP != kF32 && H >= 256 && GMC_WIDE_WAVES == 8);
    static constexpr int W = GROUPS ? 8 : kWaves;
    static constexpr int THREADS = 64 * W;
    static constexpr int NT = H / 32;                       // row tiles of a hidden layer
    static constexpr int RTW = NT / W;                      // row tiles per wave
    static constexpr int RPG = NT / 8;                      // row tiles per wave (two-group schedule)
    static constexpr int NKB1 = 16 / kb_width(P1);
    static constexpr int NKBH = H / kb_width(PH);
    static constexpr int NKB5 = H / kb_width(P5);
    static constexpr int RP = RTW >= 4 ? RTW / 2 : 1;       // row tiles per pass
    static constexpr int NP = RTW / RP;                     // row passes per layer
    // Cross-layer pipelining: pass p of wave w computes row tiles p * NT / 2 + w * RP + r, so
    // the first passes of all waves fill the first half of the consumer's k-blocks and the
    // second passes the other half; each half must be whole k-blocks.
    static constexpr bool PIPE = !GROUPS && NP == 2 && NKBH % 2 == 0 && NKB5 % 2 == 0;
    static constexpr int GH = (PIPE || GROUPS) ? NKBH / 2 : 1;
    static constexpr int G5 = (PIPE || GROUPS) ? NKB5 / 2 : 1;
    static constexpr int WPK = words_per_unit(PH) > words_per_unit(P5) ? words_per_unit(PH) : words_per_unit(P5);
    static constexpr int CT = TM / 32;                      // sample column tiles of a tile
    static constexpr int LDS_ACT = TM * ACT_STRIDE;
    static constexpr int LDS_IN = TM * IN_STRIDE;
    static constexpr int LDS_BYTES = LDS_ACT + LDS_IN + (5 + 6 + 5 + 5) * TM * 4;
};

template <int MP, int H, int RK, int TM>
__global__ __launch_bounds__((Cfg<MP, H, TM>::THREADS), 1) void mlp_ode_kernel(MlpParams p)
{
    using C = Cfg<MP, H, TM>;
    static_assert(TM == kTileM || (C::GROUPS && (TM == kSmallTileM || TM == kMidTileM)),
                  "smaller tiles are built for the two-group schedule");
    static_assert(C::LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(C::RTW >= 1 && C::NT % C::W == 0, "row tiles must split evenly over the waves");
    static_assert(C::GROUPS || C::PIPE || C::W == TM / 32,
                  "the layer-by-layer path maps one wave per column tile in layer 5");
    static_assert(!C::GROUPS || (C::RPG >= 1 && C::NKBH % 2 == 0 && C::NKB5 % 2 == 0),
                  "two-group schedule: each group's rows fill whole k-blocks of the consumer");
    __shared__ __attribute__((aligned(16))) char smem[C::LDS_BYTES];
    char *act = smem;
    char *in0 = smem + C::LDS_ACT;
    float *xs = (float *)(smem + C::LDS_ACT + C::LDS_IN);   // [5][128] ODE state
    float *cf = xs + 5 * TM;                              // [6][128] condition features
    float *ksum = cf + 6 * TM;                            // [5][128] RK4 stage sum
    float *vout = ksum + 5 * TM;                          // [5][128] last network output

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    // samples to process: the launch's own count, or one the device holds (a captured graph
    // sized for a bucket of counts); noise and raw keep the row stride p.n
    const int64_t n_items = p.n_dev ? (int64_t)*p.n_dev : p.n;
    if constexpr (TM != kTileM) {
        if (p.n_dev_large) {
            const bool large = n_items > p.small_max;
            if (blockIdx.x == 0 && threadIdx.x == 0) *p.n_dev_large = large ? (unsigned long long)n_items : 0ull;
            if (large) return;
        }
    }
    const int64_t ntiles = (n_items + TM - 1) / TM;
    const float dt = 1.0f / (float)p.K;
    constexpr bool rk4 = (RK == 1);
    const int nevals = rk4 ? 4 * p.K : p.K;
    // Euler: the lane that holds output d of sample sn applies x += dt v at once.  Classic RK4:
    // the output goes to vout; before the next evaluation the thread of sample tid forms the
    // stage input (stages at t, t + dt/2, t + dt/2, t + dt take x, x + dt/2 k1, x + dt/2 k2,
    // x + dt k3) and after the fourth stage x += dt/6 (k1 + 2 k2 + 2 k3 + k4).
    auto emit = [&](int d, int sn, float v) {
        const int o = d * TM + sn;
        if constexpr (rk4) vout[o] = v;
        else xs[o] += v * dt;
    };
    auto advance = [&](int e, float xi[5]) {
        const int stage = e & 3;
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            const int o = d * TM + tid;
            const float v = vout[o];
            if (stage < 3) {
                ksum[o] = stage == 0 ? v : ksum[o] + 2.0f * v;
                xi[d] = xs[o] + (stage == 2 ? dt : 0.5f * dt) * v;
            } else {
                xi[d] = xs[o] = xs[o] + (dt * (1.0f / 6.0f)) * (ksum[o] + v);
            }
        }
    };
    const int T0 = wave * C::RTW;                    // first row tile (layer-by-layer path)
    const int TX = wave * C::RP, TY = C::NT / 2 + wave * C::RP;   // pass row tiles (pipelined path)

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * TM;
        if (tid < TM) {
            const int64_t i = base + tid;
            float z[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            float lt = 0.f, cc = 0.f, yy = 0.5f, ss = 0.f, xx = 0.5f, co = 1.f, la = 0.f;
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
                else if (p.omega_x) la = p.omega_x[i];     // XY model: fifth feature omega_x
                if (p.noise) {
#pragma unroll
                    for (int d = 0; d < 5; ++d) z[d] = p.noise[d * p.n + i];
                } else {
                    normal5(p.keys ? p.keys[i] : p.seed, p.ids ? p.ids[i] : p.id_base + (uint64_t)i, z);
                }
            }
#pragma unroll
            for (int d = 0; d < 5; ++d) xs[d * TM + tid] = z[d];
            // boundary model: (ln tau, c, 2 y_in - 1, sin th), rectangular cells add ln A, an
            // XY-geometry model the entry direction's in-plane x component omega_x;
            // internal model: (ln tau, c, 2 x - 1, 2 y - 1, cos phi, sin phi)
            cf[0 * TM + tid] = lt;
            cf[1 * TM + tid] = cc;
            if (p.n_cond == 6) {
                cf[2 * TM + tid] = 2.0f * xx - 1.0f;
                cf[3 * TM + tid] = 2.0f * yy - 1.0f;
                cf[4 * TM + tid] = co;
                cf[5 * TM + tid] = ss;
            } else {
                cf[2 * TM + tid] = 2.0f * yy - 1.0f;
                cf[3 * TM + tid] = ss;
                cf[4 * TM + tid] = la;
                cf[5 * TM + tid] = 0.0f;
            }
        }
        __syncthreads();

        // Two-group schedule: the layer-5 lanes apply the integrator's update (Euler step, RK4
        // stage) and write the next input row themselves, so the input row is assembled here
        // only for the first evaluation.
        constexpr bool fold = C::GROUPS;
        for (int e = 0; e < nevals; ++e) {
            const int stage = rk4 ? (e & 3) : 0;
            const int k = rk4 ? (e >> 2) : e;
            const float t = ((float)k + (stage == 0 ? 0.0f : (stage == 3 ? 1.0f : 0.5f))) * dt;
            // layer-1 input row of sample tid: [x0..x4, t, ln tau, c, 2y-1, sin th, 0 x 6]
            if ((!fold || e == 0) && tid < TM) {
                float v[16];
                if (!rk4 || e == 0) {
#pragma unroll
                    for (int d = 0; d < 5; ++d) v[d] = xs[d * TM + tid];
                } else {
                    advance(e - 1, v);
                }
                v[5] = t;
#pragma unroll
                for (int d = 0; d < 6; ++d) v[6 + d] = cf[d * TM + tid];   // zero past n_cond
#pragma unroll
                for (int d = 12; d < 16; ++d) v[d] = 0.0f;
                char *row = in0 + tid * C::IN_STRIDE;
                if constexpr (C::P1 == kF32) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *(f32x4 *)(row + 16 * q) = f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
                } else {
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        *(u32x4 *)(row + 16 * q) =
                            u32x4{pack_bf16(v[8 * q], v[8 * q + 1]), pack_bf16(v[8 * q + 2], v[8 * q + 3]),
                                  pack_bf16(v[8 * q + 4], v[8 * q + 5]), pack_bf16(v[8 * q + 6], v[8 * q + 7])};
                }
            }
            if (!fold || e == 0) __syncthreads();

            if constexpr (C::GROUPS) {
                // Two-group schedule.  Per hidden layer, three barrier-separated phases:
                //   P1: group 0 multiplies over the k-blocks of the first half of the input
                //       features; group 1 runs the epilogue of its previous-layer rows (layer 1
                //       included) and writes them over the second half (nobody reads it in P1)
                //   P2: group 0 over the second half; group 1 over the first half
                //   P3: group 0 runs its epilogue into the first half; group 1 over the
                //       second half
                // Every accumulator sums its k-blocks in natural order.
                constexpr int RG = C::RPG;
                // FP8 models: the last hidden layer writes BF16, two bytes per feature, whose
                // first half would cover the FP8 second half that group 1 still reads in P3.
                // Its outputs are therefore stored with the two halves swapped (row tile
                // T -> T ^ NT/2) and layer 5 reads k-block kb from position kb ^ NKB5/2.
                constexpr int XT = (C::PH != C::P5) ? C::NT / 2 : 0;
                constexpr int SW5 = (C::PH != C::P5) ? C::NKB5 / 2 : 0;
                const int grp = wave >> 2, wg = wave & 3;
                const int TB = grp * (C::NT / 2) + wg * RG;       // first row tile of this wave
                f32x16 acc[RG][C::CT];
                // SiLU epilogue of accumulator tiles a[r][c] (row tile T0 + r, column tile c0 + c)
                // into the activation tile, row tile index xor xt
                auto drain_tiles = [&](auto POC, auto &a, int T0, int c0, float osc, float inv, int xt) {
                    constexpr int PO = decltype(POC)::value;
                    using A = std::remove_reference_t<decltype(a)>;
                    constexpr int RX = std::extent_v<A, 0>, CX = std::extent_v<A, 1>;
#if GMC_DRAIN_PIPE
                    drain_pipe<PO, C::SCALE, RX * CX>(
                        [&](auto I) {
                            constexpr int i = decltype(I)::value;
                            return a[(i / 16) / CX][(i / 16) % CX][i % 16];
                        },
                        osc, inv,
                        [&](auto TT, const uint32_t *wd) {
                            constexpr int tt = decltype(TT)::value;
                            store_tile<PO>(wd, (T0 + tt / CX) ^ xt, c0 + tt % CX, act, C::ACT_STRIDE, lane);
                        });
                    return;
#endif
                    sfor<RX * CX>([&](auto TC) {
                        constexpr int r = decltype(TC)::value / CX, c = decltype(TC)::value % CX;
                        uint32_t wd[4 * words_per_unit(PO)];
                        epi_tile<PO, C::SCALE>(a[r][c], osc, inv, wd);
                        store_tile<PO>(wd, (T0 + r) ^ xt, c0 + c, act, C::ACT_STRIDE, lane);
                    });
                };
                auto drain = [&](auto POC, float osc, float inv, int xt = 0) {
                    constexpr int PO = decltype(POC)::value;
                    constexpr int WPU = words_per_unit(PO);
#if GMC_DRAIN_PIPE
                    drain_pipe<PO, C::SCALE, RG * C::CT>(
                        [&](auto I) {
                            constexpr int i = decltype(I)::value;
                            return acc[(i / 16) / C::CT][(i / 16) % C::CT][i % 16];
                        },
                        osc, inv,
                        [&](auto TT, const uint32_t *wd) {
                            constexpr int tt = decltype(TT)::value;
                            store_tile<PO>(wd, (TB + tt / C::CT) ^ xt, tt % C::CT, act, C::ACT_STRIDE, lane);
                        });
                    return;
#endif
                    sfor<RG * C::CT>([&](auto TC) {
                        constexpr int r = decltype(TC)::value / C::CT, c = decltype(TC)::value % C::CT;
                        uint32_t wd[4 * WPU];
                        epi_tile<PO, C::SCALE>(acc[r][c], osc, inv, wd);
                        store_tile<PO>(wd, (TB + r) ^ xt, c, act, C::ACT_STRIDE, lane);
                    });
                };
                // layer 1 (10 -> H): both groups multiply their own rows; group 0 writes them now,
                // group 1 during the first hidden layer's P1.  FP8 models (whose epilogue has
                // the most vector work) split group 0's rows between the two waves of each SIMD
                // instead: group 1 recomputes the second half of them (a single k-block of
                // MFMAs) and runs that half's epilogue.
                if constexpr (MP != kFP8 || C::CT < 4) {
                    init_bias<RG, C::CT>(acc, make_rsrc(p.bias[0], p.bias_bytes[0]), TB, lane);
                    mma_seq<C::P1, RG, C::CT, C::NKB1, C::NKB1, MapAll>(acc, make_rsrc(p.wA[0], p.wA_bytes[0]), TB,
                                                                    in0, C::IN_STRIDE, 0, lane, [](auto) {});
                    if (grp == 0) drain(std::integral_constant<int, C::PH>{}, p.oscale[0], p.inv_in_scale[1]);
                } else {
                    constexpr int RS = RG >= 2 ? RG / 2 : 1;       // row tiles of each share
                    constexpr int CS = RG >= 2 ? 4 : 2;            // column tiles of each share
                    constexpr int R_OFF = RG >= 2 ? RG / 2 : 0, C_OFF = RG >= 2 ? 0 : 2;
                    const Rsrc w0 = make_rsrc(p.wA[0], p.wA_bytes[0]), b0 = make_rsrc(p.bias[0], p.bias_bytes[0]);
                    f32x16 part[RS][CS];
                    const int TS0 = wg * RG + (grp == 0 ? 0 : R_OFF), CS0 = (grp == 0) ? 0 : C_OFF;
                    if (grp != 0) {
                        init_bias<RG, C::CT>(acc, b0, TB, lane);
                        mma_seq<C::P1, RG, C::CT, C::NKB1, C::NKB1, MapAll>(acc, w0, TB, in0, C::IN_STRIDE, 0, lane,
                                                                        [](auto) {});
                    }
                    init_bias<RS, CS>(part, b0, TS0, lane);
                    mma_seq<C::P1, RS, CS, C::NKB1, C::NKB1, MapAll>(part, w0, TS0, in0, C::IN_STRIDE, CS0, lane,
                                                                     [](auto) {});
                    drain_tiles(std::integral_constant<int, C::PH>{}, part, TS0, CS0, p.oscale[0],
                                p.inv_in_scale[1], 0);
                }
                __syncthreads();
                auto hidden = [&](int l, auto OUTP) {
                    const Rsrc wl = make_rsrc(p.wA[l], p.wA_bytes[l]), bl = make_rsrc(p.bias[l], p.bias_bytes[l]);
                    const int sc = (C::PH == kFP8) ? p.mscale[l] : 127;
                    if (grp == 0) {
                        init_bias<RG, C::CT>(acc, bl, TB, lane);
                        mma_seq<C::PH, RG, C::CT, C::NKBH, C::NKBH / 2, MapHalf0<C::GH>>(
                            acc, wl, TB, act, C::ACT_STRIDE, 0, lane, [](auto) {}, sc);
                    } else {
                        drain(std::integral_constant<int, C::PH>{}, p.oscale[l - 1], p.inv_in_scale[l]);
                    }
                    __syncthreads();
                    if (grp == 0) {
                        mma_seq<C::PH, RG, C::CT, C::NKBH, C::NKBH / 2, MapHalf1<C::GH>>(
                            acc, wl, TB, act, C::ACT_STRIDE, 0, lane, [](auto) {}, sc);
                    } else {
                        init_bias<RG, C::CT>(acc, bl, TB, lane);
                        mma_seq<C::PH, RG, C::CT, C::NKBH, C::NKBH / 2, MapHalf0<C::GH>>(
                            acc, wl, TB, act, C::ACT_STRIDE, 0, lane, [](auto) {}, sc);
                    }
                    __syncthreads();
                    if (grp == 0) {
                        drain(OUTP, p.oscale[l], (l < 3) ? p.inv_in_scale[l + 1] : 1.0f,
                              decltype(OUTP)::value != C::PH ? XT : 0);
                    } else {
                        mma_seq<C::PH, RG, C::CT, C::NKBH, C::NKBH / 2, MapHalf1<C::GH>>(
                            acc, wl, TB, act, C::ACT_STRIDE, 0, lane, [](auto) {}, sc);
                    }
                    __syncthreads();
                };
                constexpr int NSAME = (C::PH == C::P5) ? 3 : 2;
#pragma unroll 1
                for (int l = 1; l <= NSAME; ++l) hidden(l, std::integral_constant<int, C::PH>{});
                if constexpr (NSAME == 2) hidden(3, std::integral_constant<int, C::P5>{});
                f32x16 out[1][1];
                const Rsrc w4 = make_rsrc(p.wA[4], p.wA_bytes[4]);
                // layer 5 (5 x H): group 0 wave w owns sample column tile w (small tiles: the
                // waves w < CT); group 1 writes its layer-4 rows meanwhile
                const bool l5 = (grp == 0) && (C::CT == 4 || wg < C::CT);
                if (l5) {
                    init_bias<1, 1>(out, make_rsrc(p.bias[4], p.bias_bytes[4]), 0, lane);
                    mma_seq<C::P5, 1, 1, C::NKB5, C::NKB5 / 2, MapHalf0<C::G5>, 0, SW5>(
                        out, w4, 0, act, C::ACT_STRIDE, wg, lane, [](auto) {});
                } else if (grp != 0) {
                    drain(std::integral_constant<int, C::P5>{}, p.oscale[3], 1.0f, XT);
                }
                __syncthreads();
                if (l5) {
                    mma_seq<C::P5, 1, 1, C::NKB5, C::NKB5 / 2, MapHalf1<C::G5>, 0, SW5>(
                        out, w4, 0, act, C::ACT_STRIDE, wg, lane, [](auto) {});
                    const int sn = wg * 32 + (lane & 31);
                    if constexpr (fold && !rk4) {
                        // x += dt v, then the next input row's x (and t) in BF16
                        char *row = in0 + sn * C::IN_STRIDE;
                        if (lane < 32) {
                            float x[4];
#pragma unroll
                            for (int d = 0; d < 4; ++d) {
                                x[d] = xs[d * TM + sn] + out[0][0][d] * dt;
                                xs[d * TM + sn] = x[d];
                            }
                            *(u32x2 *)row = u32x2{pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3])};
                        } else {
                            const float x4 = xs[4 * TM + sn] + out[0][0][0] * dt;
                            xs[4 * TM + sn] = x4;
                            *(uint32_t *)(row + 8) = pack_bf16(x4, (float)(e + 1) * dt);
                        }
                    } else if constexpr (fold) {
                        // RK4 (the arithmetic of advance): stages 0..2 add v to the stage sum
                        // and give the next stage's input, stage 3 finishes the step; then the
                        // next input row's x (and t) in BF16
                        auto update = [&](int d, float v) {
                            const int o = d * TM + sn;
                            if (stage < 3) {
                                ksum[o] = stage == 0 ? v : ksum[o] + 2.0f * v;
                                return xs[o] + (stage == 2 ? dt : 0.5f * dt) * v;
                            }
                            return xs[o] = xs[o] + (dt * (1.0f / 6.0f)) * (ksum[o] + v);
                        };
                        const int e1 = e + 1, st1 = e1 & 3;
                        const float t1 = ((float)(e1 >> 2) + (st1 == 0 ? 0.0f : (st1 == 3 ? 1.0f : 0.5f))) * dt;
                        char *row = in0 + sn * C::IN_STRIDE;
                        if (lane < 32) {
                            float x[4];
#pragma unroll
                            for (int d = 0; d < 4; ++d) x[d] = update(d, out[0][0][d]);
                            *(u32x2 *)row = u32x2{pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3])};
                        } else {
                            const float x4 = update(4, out[0][0][0]);
                            *(uint32_t *)(row + 8) = pack_bf16(x4, t1);
                        }
                    } else if (lane < 32) {
#pragma unroll
                        for (int d = 0; d < 4; ++d) emit(d, sn, out[0][0][d]);
                    } else {
                        emit(4, sn, out[0][0][0]);
                    }
                }
                __syncthreads();
                continue;
            }

            if constexpr (C::PIPE) {
                // Cross-layer pipeline.  X holds a layer's first row pass, Y its second.  Each
                // layer's second-pass epilogue runs inside the next layer's MFMA loop over the
                // k-blocks holding first-pass outputs (already in LDS); its results are stored
                // and the remaining k-blocks follow after a barrier.
                constexpr int RP = C::RP;
                f32x16 X[RP][4], Y[RP][4];
                uint32_t pk[RP * 16 * C::WPK];
                const Rsrc w0 = make_rsrc(p.wA[0], p.wA_bytes[0]), b0 = make_rsrc(p.bias[0], p.bias_bytes[0]);
                init_bias<RP, 4>(X, b0, TX, lane);
                mma_seq<C::P1, RP, 4, C::NKB1, C::NKB1, MapAll>(X, w0, TX, in0, C::IN_STRIDE, 0, lane, [](auto) {});
                init_bias<RP, 4>(Y, b0, TY, lane);
                mma_seq<C::P1, RP, 4, C::NKB1, C::NKB1, MapAll>(Y, w0, TY, in0, C::IN_STRIDE, 0, lane, [&](auto J) {
                    drain_step<C::PH, C::SCALE, RP, C::NKB1, decltype(J)::value>(X, pk, p.oscale[0], p.inv_in_scale[1]);
                });
                store_pass<C::PH, RP>(pk, TX, act, C::ACT_STRIDE, lane);
                __syncthreads();
                auto hidden = [&](int l, auto OUTP) {
                    constexpr int PO = decltype(OUTP)::value;
                    const Rsrc wl = make_rsrc(p.wA[l], p.wA_bytes[l]), bl = make_rsrc(p.bias[l], p.bias_bytes[l]);
                    const float osc_prev = p.oscale[l - 1], inv_prev = p.inv_in_scale[l];
                    const float osc = p.oscale[l], inv = (l < 3) ? p.inv_in_scale[l + 1] : 1.0f;
                    const int sc = (C::PH == kFP8) ? p.mscale[l] : 127;
                    init_bias<RP, 4>(X, bl, TX, lane);
                    mma_seq<C::PH, RP, 4, C::NKBH, C::NKBH / 2, MapHalf0<C::GH>, GMC_VPM_A>(
                        X, wl, TX, act, C::ACT_STRIDE, 0, lane, [&](auto J) {
                            drain_step<C::PH, C::SCALE, RP, C::NKBH / 2, decltype(J)::value>(Y, pk, osc_prev, inv_prev);
                        }, sc);
                    store_pass<C::PH, RP>(pk, TY, act, C::ACT_STRIDE, lane);
                    __syncthreads();
                    mma_seq<C::PH, RP, 4, C::NKBH, C::NKBH / 2, MapHalf1<C::GH>>(
                        X, wl, TX, act, C::ACT_STRIDE, 0, lane, [](auto) {}, sc);
                    init_bias<RP, 4>(Y, bl, TY, lane);
                    mma_seq<C::PH, RP, 4, C::NKBH, C::NKBH, MapAll, GMC_VPM_P>(
                        Y, wl, TY, act, C::ACT_STRIDE, 0, lane, [&](auto J) {
                            drain_step<PO, C::SCALE, RP, C::NKBH, decltype(J)::value>(X, pk, osc, inv);
                        }, sc);
                    __syncthreads();
                    store_pass<PO, RP>(pk, TX, act, C::ACT_STRIDE, lane);
                    __syncthreads();
                };
                constexpr int NSAME = (C::PH == C::P5) ? 3 : 2;
#pragma unroll 1
                for (int l = 1; l <= NSAME; ++l) hidden(l, std::integral_constant<int, C::PH>{});
                if constexpr (NSAME == 2) hidden(3, std::integral_constant<int, C::P5>{});
                // layer 5 (5 x H, rows padded to one tile) over the first-pass k-blocks while
                // layer 4's second pass drains; wave w < 4 owns sample column tile w, further
                // waves only drain
                constexpr int CT5 = TM / 32;
                f32x16 out[1][1];
                const Rsrc w4 = make_rsrc(p.wA[4], p.wA_bytes[4]);
                auto drain4 = [&](auto J) {
                    drain_step<C::P5, C::SCALE, RP, C::NKB5 / 2, decltype(J)::value>(Y, pk, p.oscale[3], 1.0f);
                };
                if (C::W == CT5 || wave < CT5) {
                    init_bias<1, 1>(out, make_rsrc(p.bias[4], p.bias_bytes[4]), 0, lane);
                    mma_seq<C::P5, 1, 1, C::NKB5, C::NKB5 / 2, MapHalf0<C::G5>, GMC_VPM_5>(
                        out, w4, 0, act, C::ACT_STRIDE, wave, lane, drain4);
                } else {
                    sfor<C::NKB5 / 2>(drain4);
                }
                store_pass<C::P5, RP>(pk, TY, act, C::ACT_STRIDE, lane);
                __syncthreads();
                if (C::W == CT5 || wave < CT5) {
                    mma_seq<C::P5, 1, 1, C::NKB5, C::NKB5 / 2, MapHalf1<C::G5>>(
                        out, w4, 0, act, C::ACT_STRIDE, wave, lane, [](auto) {});
                    const int sn = wave * 32 + (lane & 31);
                    if (lane < 32) {
#pragma unroll
                        for (int d = 0; d < 4; ++d) emit(d, sn, out[0][0][d]);
                    } else {
                        emit(4, sn, out[0][0][0]);
                    }
                }
                __syncthreads();
                continue;
            }

            // layer 1: 10 -> H (reads in0, writes the activation tile: no barrier before writing)
            dense_silu<C::P1, C::PH, C::RTW, C::NKB1, C::SCALE, false>(
                make_rsrc(p.wA[0], p.wA_bytes[0]), make_rsrc(p.bias[0], p.bias_bytes[0]), T0, in0, C::IN_STRIDE, act, C::ACT_STRIDE, lane,
                p.oscale[0], p.inv_in_scale[1]);
            __syncthreads();
            // hidden layers 2..4: H -> H, in place.  One code instance in a runtime loop (layers
            // whose output feeds an operand of the same type as their input); an FP8 model's
            // last hidden layer writes BF16 for the output layer and is a second instance.
            constexpr int NSAME = (C::PH == C::P5) ? 3 : 2;
#pragma unroll 1
            for (int l = 1; l <= NSAME; ++l) {
                dense_silu<C::PH, C::PH, C::RTW, C::NKBH, C::SCALE, true>(
                    make_rsrc(p.wA[l], p.wA_bytes[l]), make_rsrc(p.bias[l], p.bias_bytes[l]), T0,
                    act, C::ACT_STRIDE, act, C::ACT_STRIDE, lane, p.oscale[l],
                    l < 3 ? p.inv_in_scale[l + 1] : 1.0f, (C::PH == kFP8) ? p.mscale[l] : 127);
                __syncthreads();
            }
            if constexpr (NSAME == 2) {
                dense_silu<C::PH, C::P5, C::RTW, C::NKBH, C::SCALE, true>(
                    make_rsrc(p.wA[3], p.wA_bytes[3]), make_rsrc(p.bias[3], p.bias_bytes[3]), T0,
                    act, C::ACT_STRIDE, act, C::ACT_STRIDE, lane, p.oscale[3], 1.0f,
                    (C::PH == kFP8) ? p.mscale[3] : 127);
                __syncthreads();
            }
            // layer 5: H -> 5 (rows padded to 32); wave w handles sample column tile w
            {
                f32x16 out[1][1];
                init_bias<1, 1>(out, make_rsrc(p.bias[4], p.bias_bytes[4]), 0, lane);
                mma_pass<C::P5, 1, 1, C::NKB5>(out, make_rsrc(p.wA[4], p.wA_bytes[4]), 0, act,
                                               C::ACT_STRIDE, wave, lane, [](auto) {});
                const int sn = wave * 32 + (lane & 31);
                if (lane < 32) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) emit(d, sn, out[0][0][d]);
                } else {
                    emit(4, sn, out[0][0][0]);
                }
            }
            __syncthreads();
        }

        if (tid < TM) {
            const int64_t i = base + tid;
            float xk[5];
            if constexpr (rk4 && !fold) {
                advance(nevals - 1, xk);
            } else {
#pragma unroll
                for (int d = 0; d < 5; ++d) xk[d] = xs[d * TM + tid];
            }
            if (i < n_items) {
                const float a0 = xk[0], a1 = xk[1], a2 = xk[2], a3 = xk[3], a4 = xk[4];
                if (p.raw) {
                    p.raw[0 * p.n + i] = a0;
                    p.raw[1 * p.n + i] = a1;
                    p.raw[2 * p.n + i] = a2;
                    p.raw[3 * p.n + i] = a3;
                    p.raw[4 * p.n + i] = a4;
                }
                Exit e;
                decode_exit(a0, a1, a2, a3, a4, e, p.xy != 0);
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

// Persistent workgroups per compute unit of one kernel instance.  The two-group kernels fill
// a CU's LDS and keep one.  A four-wave kernel has one wave per SIMD, which leaves the vector
// units idle while it runs matrix work and the matrix core idle during its epilogue; where
// registers and LDS leave room, several of its workgroups share a CU and their phases
// interleave (the occupancy query, at most GMC_MAX_WG_PER_CU; queried once per instance).
template <int MP, int H, int RK, int TM>
int resident_per_cu()
{
    if constexpr (Cfg<MP, H, TM>::GROUPS) {
        return 1;
    } else {
        static const int n = [] {
            int b = 1;
            const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &b, reinterpret_cast<const void *>(&mlp_ode_kernel<MP, H, RK, TM>), Cfg<MP, H, TM>::THREADS, 0);
            if (e != hipSuccess) {
                (void)hipGetLastError();   // fall back to one workgroup; keep the error off later launches
                b = 1;
            }
            return std::max(1, std::min(b, GMC_MAX_WG_PER_CU));
        }();
        return n;
    }
}

// grid: one persistent workgroup per tile of a launch of at most `bound` samples, at most
// cu x resident_per_cu
template <int MP, int H, int TM>
hipError_t launch_tiles(const MlpParams &p, int64_t bound, int cu, hipStream_t s)
{
    constexpr int threads = Cfg<MP, H, TM>::THREADS;
    const int64_t ntiles = (bound + TM - 1) / TM;
    const int per_cu = p.integrator == 1 ? resident_per_cu<MP, H, 1, TM>() : resident_per_cu<MP, H, 0, TM>();
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)cu * per_cu));
    if (p.integrator == 1) hipLaunchKernelGGL((mlp_ode_kernel<MP, H, 1, TM>), dim3(grid), dim3(threads), 0, s, p);
    else hipLaunchKernelGGL((mlp_ode_kernel<MP, H, 0, TM>), dim3(grid), dim3(threads), 0, s, p);
    return hipGetLastError();
}

// The same launch over samples [off, off + cnt) of p: every per-sample array moves by off (the
// [5][n] noise and raw arrays, whose row stride is p.n, are not used with it).
inline MlpParams sample_range(const MlpParams &p, int64_t off, int64_t cnt)
{
    MlpParams q = p;
    auto mv = [off](auto *&ptr) { if (ptr) ptr += off; };
    mv(q.log_tau); mv(q.c); mv(q.y_in); mv(q.sin_th); mv(q.x_in); mv(q.cos_phi);
    mv(q.log_aspect); mv(q.omega_x); mv(q.ids); mv(q.keys);
    mv(q.face); mv(q.pos); mv(q.dcos); mv(q.dsin); mv(q.path);
    if (!p.ids) q.id_base = p.id_base + (uint64_t)off;
    q.n = cnt;
    return q;
}

// Launches with at most kSmallTileM (kMidTileM) samples per compute unit (the tail steps of a
// transport run, small requests) take 32-sample (64-sample) tiles when the model runs the
// two-group schedule: one round of them covers the launch on every CU, and a tile's latency
// falls with its matrix work (RK4 x 12 at width 512: 0.75 ms for 32 samples, 1.6 ms for 128).
// When only the device knows the count (n_dev) and its bound p.n is larger, the choice is made
// on the device (MlpParams::n_dev_large) without a read-back; a sample's result is the same
// with every tile size.  A count known on the host whose last round of 128-sample tiles would
// hold at most 64 samples per CU runs that remainder as one round of smaller tiles.
template <int MP, int H>
hipError_t launch_one(const MlpParams &p, int cu, hipStream_t s)
{
    MlpParams q = p;
    q.n_dev_large = nullptr;
    if constexpr (Cfg<MP, H>::GROUPS) {
        const int64_t small = (int64_t)kSmallTileM * cu, mid = (int64_t)kMidTileM * cu;
        if (p.n <= small) return launch_tiles<MP, H, kSmallTileM>(q, p.n, cu, s);
        if (!p.n_dev) {
            if (p.n <= mid) return launch_tiles<MP, H, kMidTileM>(q, p.n, cu, s);
            const int64_t round = (int64_t)kTileM * cu, rem = p.n % round;
            if (!p.noise && !p.raw && rem > 0 && rem <= mid) {
                const MlpParams head = sample_range(q, 0, p.n - rem);
                const hipError_t e = launch_tiles<MP, H, kTileM>(head, head.n, cu, s);
                if (e != hipSuccess) return e;
                const MlpParams tail = sample_range(q, p.n - rem, rem);
                return rem <= small ? launch_tiles<MP, H, kSmallTileM>(tail, rem, cu, s)
                                    : launch_tiles<MP, H, kMidTileM>(tail, rem, cu, s);
            }
        } else if (p.n_dev_large) {
            // 32-sample kernel, then the 64-sample one, each handing on what it does not take
            q.n_dev_large = p.n_dev_large;
            q.small_max = small;
            hipError_t e = launch_tiles<MP, H, kSmallTileM>(q, small, cu, s);
            if (e != hipSuccess) return e;
            q.n_dev = p.n_dev_large;
            q.n_dev_large = p.n <= mid ? nullptr : p.n_dev_large + 1;
            q.small_max = mid;
            e = launch_tiles<MP, H, kMidTileM>(q, std::min<int64_t>(p.n, mid), cu, s);
            if (e != hipSuccess || p.n <= mid) return e;
            q.n_dev = p.n_dev_large + 1;
            q.n_dev_large = nullptr;
        }
    }
    return launch_tiles<MP, H, kTileM>(q, p.n, cu, s);
}

}  // namespace

bool mlp_supported(int prec, int hidden)
{
    if (prec == kF32) return hidden == 128 || hidden == 256;
    if (prec == kBF16 || prec == kFP8) return hidden == 128 || hidden == 256 || hidden == 512;
    return false;
}

template <int MP, int H>
void prepare_one()
{
    (void)resident_per_cu<MP, H, 0, kTileM>();
    (void)resident_per_cu<MP, H, 1, kTileM>();
}

void mlp_prepare(int prec, int hidden)
{
    switch (prec * 1000 + hidden) {
    case kF32 * 1000 + 128: prepare_one<kF32, 128>(); break;
    case kF32 * 1000 + 256: prepare_one<kF32, 256>(); break;
    case kBF16 * 1000 + 128: prepare_one<kBF16, 128>(); break;
    case kBF16 * 1000 + 256: prepare_one<kBF16, 256>(); break;
    case kBF16 * 1000 + 512: prepare_one<kBF16, 512>(); break;
    case kFP8 * 1000 + 128: prepare_one<kFP8, 128>(); break;
    case kFP8 * 1000 + 256: prepare_one<kFP8, 256>(); break;
    case kFP8 * 1000 + 512: prepare_one<kFP8, 512>(); break;
    default: break;
    }
}

hipError_t launch_mlp_ode(int prec, int hidden, const MlpParams &p, int cu, hipStream_t s)
{
    if (p.net == 1) return launch_film_ode(prec, hidden, p, cu, s);
    switch (prec * 1000 + hidden) {
    case kF32 * 1000 + 128: return launch_one<kF32, 128>(p, cu, s);
    case kF32 * 1000 + 256: return launch_one<kF32, 256>(p, cu, s);
    case kBF16 * 1000 + 128: return launch_one<kBF16, 128>(p, cu, s);
    case kBF16 * 1000 + 256: return launch_one<kBF16, 256>(p, cu, s);
    case kBF16 * 1000 + 512: return launch_one<kBF16, 512>(p, cu, s);
    case kFP8 * 1000 + 128: return launch_one<kFP8, 128>(p, cu, s);
    case kFP8 * 1000 + 256: return launch_one<kFP8, 256>(p, cu, s);
    case kFP8 * 1000 + 512: return launch_one<kFP8, 512>(p, cu, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gmc
