// Fused sampler for the residual velocity network with adaptive modulation (paper: section
// "Network Architecture and Inputs" -- learned embeddings of the flow time and the condition,
// residual blocks modulated by the physical context; section "Conditional Flow Matching",
// eq. 8 -- the ODE, integrated by explicit Euler or classic RK4; eq. 11 -- decoding).
//
// The network (the library's reading of a section whose layer details are not given):
//   u   = [x (5), phi(t) (8), condition (4..6)],  phi = sin, cos of pi 2^j t, j = 0..3
//   h0  = W_in u + b_in
//   e   = SiLU(W_e [phi, condition] + b_e)                          (width 32)
//   h  <- h + SiLU((1 + G_j e + g_j) * (A_j h + a_j) + (S_j e + s_j)),  j = 1..3
//   v   = W_o h + b_o
//
// One persistent workgroup per CU carries a tile of 128 samples through all evaluations; LDS
// holds the input row tile (32 features), the embedding tile (32 features) and the residual
// stream h (128 x H), all in the operand precision, and the ODE state.  The input layer and the
// embedding are MFMA contractions over the input row tile.
//   * BF16, H >= 256: two groups of four waves (two waves per SIMD).  Group 0 owns the first
//     half of a block's output rows, group 1 the second; per block, three barrier-separated
//     phases pair one group's matrix k-loop with the other group's epilogue on the same SIMDs
//     (the plain sampler's schedule).  A group's epilogue (two 32 -> H modulation
//     contractions over the embedding tile, the modulated SiLU, the residual add, the store)
//     writes rows of h that only it reads at that time, and reads the residual from the rows
//     it overwrites, which still hold the block's input.
//   * FP32 and H = 128: four waves, one per SIMD: a block's main H x H contraction for all of
//     the wave's row tiles, a barrier, then per accumulator tile the modulation contractions,
//     issued one tile ahead so they overlap the previous tile's vector work, the modulated
//     SiLU, the residual add and the store; a barrier.
//   * The output layer: four waves, one sample column tile each, and the ODE update.
// The weights of every layer are arranged on the host in MFMA fragment order; the columns of
// the layers that read an accumulator-written tile are permuted to the order the producing
// accumulators stored (phys_to_feature), the "1 +" of the scale is folded into its bias.
#include <algorithm>

#include "gmc_mma.hpp"

namespace gmc {
namespace {

template <int MP, int H>
struct FilmCfg {
    static constexpr int EB = elem_bytes(MP);
    static constexpr int ACT_STRIDE = H * EB + 16;          // +16 B: conflict-free row reads
    static constexpr int IN_STRIDE = kFilmIn * EB + 16;
    static constexpr int EMB_STRIDE = kFilmEmb * EB + 16;
    // Two-group schedule (BF16, H >= 256): eight waves, two per SIMD; group 0 owns the first
    // half of every block's output rows, group 1 the second half, and while one group runs its
    // matrix k-loop the other runs its epilogue on the same SIMDs.
    static constexpr bool GROUPS = (MP == kBF16 && H >= 256);
    static constexpr int W = GROUPS ? 8 : 4;                 // waves
    static constexpr int THREADS = 64 * W;
    static constexpr int NT = H / 32;                        // row tiles of a hidden layer
    static constexpr int RTW = GROUPS ? NT / 8 : NT / W;     // row tiles per wave
    static constexpr int NKB_IN = kFilmIn / kb_width(MP);
    static constexpr int NKB_E = kFilmEmb / kb_width(MP);
    static constexpr int NKBH = H / kb_width(MP);
    static constexpr int WPT = 4 * words_per_unit(MP);       // packed words per accumulator tile
    static constexpr int LDS_ACT = kTileM * ACT_STRIDE;
    static constexpr int LDS_IN = kTileM * IN_STRIDE;
    static constexpr int LDS_EMB = kTileM * EMB_STRIDE;
    static constexpr int LDS_BYTES = LDS_ACT + LDS_IN + LDS_EMB + 3 * 5 * kTileM * 4;
};

// Reads back the 16 values of accumulator tile (row tile T, column tile c) of this lane from an
// LDS activation tile written by store_tile<PO> (the same positions, the same value order).
template <int PO>
__device__ __forceinline__ void load_tile(float *v, int T, int c, const char *act, int stride, int lane)
{
    const int h = lane >> 5, n = lane & 31;
    const char *row = act + (c * 32 + n) * stride;
    if constexpr (PO == kF32) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const f32x4 q = *(const f32x4 *)(row + ((4 * T + g) * 8 + 4 * h) * 4);
            v[4 * g + 0] = q.x;
            v[4 * g + 1] = q.y;
            v[4 * g + 2] = q.z;
            v[4 * g + 3] = q.w;
        }
    } else {
        static_assert(PO == kBF16, "the residual network's operands are FP32 or BF16");
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const u32x4 w = *(const u32x4 *)(row + ((2 * T + q) * 16 + 8 * h) * 2);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                v[8 * q + 2 * m] = __builtin_bit_cast(float, w[m] << 16);
                v[8 * q + 2 * m + 1] = __builtin_bit_cast(float, w[m] & 0xFFFF0000u);
            }
        }
    }
}

// Packs 16 accumulator-order values of one tile into the words store_tile<PO> takes.
template <int PO>
__device__ __forceinline__ void pack_tile(const float *y, uint32_t *w)
{
    if constexpr (PO == kF32) {
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = __builtin_bit_cast(uint32_t, y[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = pack_bf16(y[2 * i], y[2 * i + 1]);
    }
}

template <int MP, int H, int RK>
__global__ __launch_bounds__((FilmCfg<MP, H>::THREADS), 1) void film_ode_kernel(MlpParams p)
{
    using C = FilmCfg<MP, H>;
    static_assert(C::LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(C::RTW >= 1 && C::NT % C::W == 0, "row tiles must split evenly over the waves");
    static_assert(!C::GROUPS || C::NKBH % 2 == 0, "two-group schedule: each group's rows fill whole k-blocks");
    __shared__ __attribute__((aligned(16))) char smem[C::LDS_BYTES];
    char *act = smem;
    char *in0 = smem + C::LDS_ACT;
    char *emb = in0 + C::LDS_IN;
    float *xs = (float *)(emb + C::LDS_EMB);     // [5][128] ODE state
    float *ksum = xs + 5 * kTileM;                // [5][128] RK4 stage sum
    float *vout = ksum + 5 * kTileM;              // [5][128] last network output

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t n_items = p.n_dev ? (int64_t)*p.n_dev : p.n;
    const int64_t ntiles = (n_items + kTileM - 1) / kTileM;
    const float dt = 1.0f / (float)p.K;
    constexpr bool rk4 = (RK == 1);
    const int nevals = rk4 ? 4 * p.K : p.K;
    auto emit = [&](int d, int sn, float v) {
        const int o = d * kTileM + sn;
        if constexpr (rk4) vout[o] = v;
        else xs[o] += v * dt;
    };
    // classic RK4: stage inputs x, x + dt/2 k1, x + dt/2 k2, x + dt k3; after the fourth stage
    // x += dt/6 (k1 + 2 k2 + 2 k3 + k4) (the same steps as the plain sampler)
    auto advance = [&](int e, float xi[5]) {
        const int stage = e & 3;
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            const int o = d * kTileM + tid;
            const float v = vout[o];
            if (stage < 3) {
                ksum[o] = stage == 0 ? v : ksum[o] + 2.0f * v;
                xi[d] = xs[o] + (stage == 2 ? dt : 0.5f * dt) * v;
            } else {
                xi[d] = xs[o] = xs[o] + (dt * (1.0f / 6.0f)) * (ksum[o] + v);
            }
        }
    };
    const int T0 = wave * C::RTW;
    auto nohook = [](auto) {};

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * kTileM;
        float cv[6];
        if (tid < kTileM) {
            float z[5];
            sampler_inputs(p, base + tid, n_items, z, cv);
#pragma unroll
            for (int d = 0; d < 5; ++d) xs[d * kTileM + tid] = z[d];
        }
        __syncthreads();

        // Two-group kernels: the output layer's lanes apply the integrator's update and write
        // the next input row's x and time features themselves, so the row is assembled here only
        // for the first evaluation.
        constexpr bool fold = C::GROUPS;
        for (int e = 0; e < nevals; ++e) {
            const int stage = rk4 ? (e & 3) : 0;
            const int k = rk4 ? (e >> 2) : e;
            const float t = ((float)k + (stage == 0 ? 0.0f : (stage == 3 ? 1.0f : 0.5f))) * dt;
            // input row of sample tid: [x0..x4, sin pi t, cos pi t, ..., cos 8 pi t, condition, 0...]
            if ((!fold || e == 0) && tid < kTileM) {
                float v[kFilmIn];
                if (!rk4 || e == 0) {
#pragma unroll
                    for (int d = 0; d < 5; ++d) v[d] = xs[d * kTileM + tid];
                } else {
                    advance(e - 1, v);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float a = (float)(1 << j) * t;       // exact: a power of two times t
                    v[5 + 2 * j] = sinpif(a);
                    v[6 + 2 * j] = cospif(a);
                }
#pragma unroll
                for (int d = 0; d < 6; ++d) v[13 + d] = cv[d];
#pragma unroll
                for (int d = 19; d < kFilmIn; ++d) v[d] = 0.0f;
                char *row = in0 + tid * C::IN_STRIDE;
                if constexpr (MP == kF32) {
#pragma unroll
                    for (int q = 0; q < kFilmIn / 4; ++q)
                        *(f32x4 *)(row + 16 * q) = f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
                } else {
#pragma unroll
                    for (int q = 0; q < kFilmIn / 8; ++q)
                        *(u32x4 *)(row + 16 * q) =
                            u32x4{pack_bf16(v[8 * q], v[8 * q + 1]), pack_bf16(v[8 * q + 2], v[8 * q + 3]),
                                  pack_bf16(v[8 * q + 4], v[8 * q + 5]), pack_bf16(v[8 * q + 6], v[8 * q + 7])};
                }
            }
            if (!fold || e == 0) __syncthreads();

            if constexpr (C::GROUPS) {
                // Two-group schedule.  Per block, three barrier-separated phases (as in the plain
                // sampler): P1 group 0 multiplies over the first half of the k-blocks (its own
                // rows of h) while group 1 runs the epilogue of its rows of the previous block;
                // P2 group 0 over the second half, group 1 over the first; P3 group 0 runs its
                // epilogue while group 1 multiplies over the second half.  A group's epilogue
                // writes rows of h only it reads meanwhile, and reads the residual from the rows
                // it overwrites, which still hold the block's input.
                constexpr int RG = C::RTW;
                constexpr int GH = C::NKBH / 2;
                const int grp = wave >> 2, wg = wave & 3;
                const int TB = grp * (C::NT / 2) + wg * RG;      // first row tile of this wave
                f32x16 acc[RG][4];
                // input layer: every wave its own rows (no activation); group 1 also the
                // embedding (wave wg: sample column tile wg)
                init_bias<RG, 4>(acc, make_rsrc(p.bias[0], p.bias_bytes[0]), TB, lane);
                mma_seq<MP, RG, 4, C::NKB_IN, C::NKB_IN, MapAll>(acc, make_rsrc(p.wA[0], p.wA_bytes[0]), TB, in0,
                                                                 C::IN_STRIDE, 0, lane, nohook);
                sfor<RG * 4>([&](auto TC) {
                    constexpr int r = decltype(TC)::value / 4, c = decltype(TC)::value % 4;
                    float y[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) y[i] = acc[r][c][i];
                    uint32_t w[C::WPT];
                    pack_tile<MP>(y, w);
                    store_tile<MP>(w, TB + r, c, act, C::ACT_STRIDE, lane);
                });
                if (grp == 1) {
                    f32x16 ea[1][1];
                    init_bias<1, 1>(ea, make_rsrc(p.bias[1], p.bias_bytes[1]), 0, lane);
                    mma_seq<MP, 1, 1, C::NKB_IN, C::NKB_IN, MapAll>(ea, make_rsrc(p.wA[1], p.wA_bytes[1]), 0, in0,
                                                                    C::IN_STRIDE, wg, lane, nohook);
                    float y[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) y[i] = silu(ea[0][0][i]);
                    uint32_t w[C::WPT];
                    pack_tile<MP>(y, w);
                    store_tile<MP>(w, 0, wg, emb, C::EMB_STRIDE, lane);
                }
                __syncthreads();
                // the epilogue of block j for this wave's tiles: the two modulation contractions
                // over the embedding tile, the modulated SiLU, the residual add, the store
                // Per row tile the scale and shift maps' weight fragments and biases are loaded
                // once and serve the four sample column tiles.
                auto epilogue = [&](int j) {
                    using M = Mma<MP>;
                    constexpr int KBB = kb_width(MP) * elem_bytes(MP);
                    const int lG = 3 + 3 * j, lS = lG + 1;
                    const Rsrc wG = make_rsrc(p.wA[lG], p.wA_bytes[lG]), bG = make_rsrc(p.bias[lG], p.bias_bytes[lG]);
                    const Rsrc wS = make_rsrc(p.wA[lS], p.wA_bytes[lS]), bS = make_rsrc(p.bias[lS], p.bias_bytes[lS]);
                    const int h = lane >> 5, n = lane & 31;
                    sfor<RG>([&](auto R) {
                        constexpr int r = decltype(R)::value;
                        const int t = __builtin_amdgcn_readfirstlane(TB + r);
                        typename M::Frag ga[C::NKB_E], sa[C::NKB_E];
#pragma unroll
                        for (int kb = 0; kb < C::NKB_E; ++kb) {
                            ga[kb] = M::load_g(wG, lane * frag_bytes(MP), (t * C::NKB_E + kb) * 64 * frag_bytes(MP));
                            sa[kb] = M::load_g(wS, lane * frag_bytes(MP), (t * C::NKB_E + kb) * 64 * frag_bytes(MP));
                        }
                        f32x16 bgv[1][1], bsv[1][1];
                        init_bias<1, 1>(bgv, bG, TB + r, lane);
                        init_bias<1, 1>(bsv, bS, TB + r, lane);
                        sfor<4>([&](auto CC) {
                            constexpr int c = decltype(CC)::value;
                            f32x16 sc = bgv[0][0], sh = bsv[0][0];
                            const char *sb = emb + (c * 32 + n) * C::EMB_STRIDE + h * (KBB / 2);
#pragma unroll
                            for (int kb = 0; kb < C::NKB_E; ++kb) {
                                const typename M::Frag b = M::load_s(sb + kb * KBB);
                                M::run(sc, ga[kb], b, 127);
                                M::run(sh, sa[kb], b, 127);
                            }
                            float hp[16], y[16];
                            load_tile<MP>(hp, TB + r, c, act, C::ACT_STRIDE, lane);
#pragma unroll
                            for (int i = 0; i < 16; ++i)
                                y[i] = hp[i] + silu(__builtin_fmaf(sc[i], acc[r][c][i], sh[i]));
                            uint32_t w[C::WPT];
                            pack_tile<MP>(y, w);
                            store_tile<MP>(w, TB + r, c, act, C::ACT_STRIDE, lane);
                        });
                    });
                };
#pragma unroll 1
                for (int j = 0; j < kFilmBlocks; ++j) {
                    const int lA = 2 + 3 * j;
                    const Rsrc wA = make_rsrc(p.wA[lA], p.wA_bytes[lA]), bA = make_rsrc(p.bias[lA], p.bias_bytes[lA]);
                    if (grp == 0) {
                        init_bias<RG, 4>(acc, bA, TB, lane);
                        mma_seq<MP, RG, 4, C::NKBH, GH, MapHalf0<GH>>(acc, wA, TB, act, C::ACT_STRIDE, 0, lane, nohook);
                    } else if (j > 0) {
                        epilogue(j - 1);
                    }
                    __syncthreads();
                    if (grp == 0) {
                        mma_seq<MP, RG, 4, C::NKBH, GH, MapHalf1<GH>>(acc, wA, TB, act, C::ACT_STRIDE, 0, lane, nohook);
                    } else {
                        init_bias<RG, 4>(acc, bA, TB, lane);
                        mma_seq<MP, RG, 4, C::NKBH, GH, MapHalf0<GH>>(acc, wA, TB, act, C::ACT_STRIDE, 0, lane, nohook);
                    }
                    __syncthreads();
                    if (grp == 0) {
                        epilogue(j);
                    } else {
                        mma_seq<MP, RG, 4, C::NKBH, GH, MapHalf1<GH>>(acc, wA, TB, act, C::ACT_STRIDE, 0, lane, nohook);
                    }
                    __syncthreads();
                }
                // output layer (5 x H, rows padded to one tile): group 0 wave wg, sample column
                // tile wg, over the first half while group 1 writes its rows of the last block
                f32x16 out[1][1];
                const Rsrc wO = make_rsrc(p.wA[kMaxLayers - 1], p.wA_bytes[kMaxLayers - 1]);
                if (grp == 0) {
                    init_bias<1, 1>(out, make_rsrc(p.bias[kMaxLayers - 1], p.bias_bytes[kMaxLayers - 1]), 0, lane);
                    mma_seq<MP, 1, 1, C::NKBH, GH, MapHalf0<GH>>(out, wO, 0, act, C::ACT_STRIDE, wg, lane, nohook);
                } else {
                    epilogue(kFilmBlocks - 1);
                }
                __syncthreads();
                if (grp == 0) {
                    mma_seq<MP, 1, 1, C::NKBH, GH, MapHalf1<GH>>(out, wO, 0, act, C::ACT_STRIDE, wg, lane, nohook);
                    const int sn = wg * 32 + (lane & 31);
                    // the integrator's update of component d of sample sn by the velocity v
                    // (the arithmetic of emit / advance); returns the next evaluation's input
                    auto update = [&](int d, float v) {
                        const int o = d * kTileM + sn;
                        if constexpr (rk4) {
                            if (stage < 3) {
                                ksum[o] = stage == 0 ? v : ksum[o] + 2.0f * v;
                                return xs[o] + (stage == 2 ? dt : 0.5f * dt) * v;
                            }
                            return xs[o] = xs[o] + (dt * (1.0f / 6.0f)) * (ksum[o] + v);
                        } else {
                            return xs[o] = xs[o] + v * dt;
                        }
                    };
                    // the next input row in BF16: x0..x3 (bytes 0-7) from lanes 0-31, x4 and the
                    // eight time features of the next evaluation's t (bytes 8-25) from lanes
                    // 32-63; the condition columns keep what the first evaluation wrote
                    char *row = in0 + sn * C::IN_STRIDE;
                    if (lane < 32) {
                        float x[4];
#pragma unroll
                        for (int d = 0; d < 4; ++d) x[d] = update(d, out[0][0][d]);
                        *(u32x2 *)row = u32x2{pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3])};
                    } else {
                        const int e1 = e + 1, st1 = rk4 ? (e1 & 3) : 0, k1 = rk4 ? (e1 >> 2) : e1;
                        const float t1 = ((float)k1 + (st1 == 0 ? 0.0f : (st1 == 3 ? 1.0f : 0.5f))) * dt;
                        float f[9];
                        f[0] = update(4, out[0][0][0]);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float a = (float)(1 << j) * t1;
                            f[1 + 2 * j] = sinpif(a);
                            f[2 + 2 * j] = cospif(a);
                        }
                        *(u32x2 *)(row + 8) = u32x2{pack_bf16(f[0], f[1]), pack_bf16(f[2], f[3])};
                        *(u32x2 *)(row + 16) = u32x2{pack_bf16(f[4], f[5]), pack_bf16(f[6], f[7])};
                        *(uint16_t *)(row + 24) = (uint16_t)(pack_bf16(f[8], 0.0f) & 0xFFFFu);
                    }
                }
                __syncthreads();
            } else {
                // embedding (wave w: sample column tile w) and input layer (the wave's row tiles):
                // both read only the input row tile
                {
                    f32x16 ea[1][1];
                    init_bias<1, 1>(ea, make_rsrc(p.bias[1], p.bias_bytes[1]), 0, lane);
                    mma_pass<MP, 1, 1, C::NKB_IN>(ea, make_rsrc(p.wA[1], p.wA_bytes[1]), 0, in0, C::IN_STRIDE,
                                                  wave, lane, nohook);
                    float y[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) y[i] = silu(ea[0][0][i]);
                    uint32_t w[C::WPT];
                    pack_tile<MP>(y, w);
                    store_tile<MP>(w, 0, wave, emb, C::EMB_STRIDE, lane);
                }
                {
                    f32x16 acc[C::RTW][4];
                    init_bias<C::RTW, 4>(acc, make_rsrc(p.bias[0], p.bias_bytes[0]), T0, lane);
                    mma_pass<MP, C::RTW, 4, C::NKB_IN>(acc, make_rsrc(p.wA[0], p.wA_bytes[0]), T0, in0,
                                                       C::IN_STRIDE, 0, lane, nohook);
                    sfor<C::RTW * 4>([&](auto TC) {
                        constexpr int r = decltype(TC)::value / 4, c = decltype(TC)::value % 4;
                        float y[16];
#pragma unroll
                        for (int i = 0; i < 16; ++i) y[i] = acc[r][c][i];
                        uint32_t w[C::WPT];
                        pack_tile<MP>(y, w);
                        store_tile<MP>(w, T0 + r, c, act, C::ACT_STRIDE, lane);
                    });
                }
                __syncthreads();

                // residual blocks
#pragma unroll 1
                for (int j = 0; j < kFilmBlocks; ++j) {
                    const int lA = 2 + 3 * j, lG = lA + 1, lS = lA + 2;
                    const Rsrc wG = make_rsrc(p.wA[lG], p.wA_bytes[lG]), bG = make_rsrc(p.bias[lG], p.bias_bytes[lG]);
                    const Rsrc wS = make_rsrc(p.wA[lS], p.wA_bytes[lS]), bS = make_rsrc(p.bias[lS], p.bias_bytes[lS]);
                    f32x16 acc[C::RTW][4];
                    init_bias<C::RTW, 4>(acc, make_rsrc(p.bias[lA], p.bias_bytes[lA]), T0, lane);
                    mma_pass<MP, C::RTW, 4, C::NKBH>(acc, make_rsrc(p.wA[lA], p.wA_bytes[lA]), T0, act,
                                                     C::ACT_STRIDE, 0, lane, nohook);
                    __syncthreads();   // every wave has read h: the block's outputs may overwrite it
                    // modulation of tile q (row tile T0 + q / 4, column tile q % 4) into slot q % 2
                    f32x16 sc[2][1][1], sh[2][1][1];
                    auto modulation = [&](auto Q) {
                        constexpr int q = decltype(Q)::value, r = q / 4, c = q % 4;
                        init_bias<1, 1>(sc[q % 2], bG, T0 + r, lane);
                        mma_pass<MP, 1, 1, C::NKB_E>(sc[q % 2], wG, T0 + r, emb, C::EMB_STRIDE, c, lane, nohook);
                        init_bias<1, 1>(sh[q % 2], bS, T0 + r, lane);
                        mma_pass<MP, 1, 1, C::NKB_E>(sh[q % 2], wS, T0 + r, emb, C::EMB_STRIDE, c, lane, nohook);
                    };
                    modulation(std::integral_constant<int, 0>{});
                    sfor<C::RTW * 4>([&](auto Q) {
                        constexpr int q = decltype(Q)::value, r = q / 4, c = q % 4;
                        if constexpr (q + 1 < C::RTW * 4) modulation(std::integral_constant<int, q + 1>{});
                        float hp[16], y[16];
                        load_tile<MP>(hp, T0 + r, c, act, C::ACT_STRIDE, lane);
#pragma unroll
                        for (int i = 0; i < 16; ++i)
                            y[i] = hp[i] + silu(__builtin_fmaf(sc[q % 2][0][0][i], acc[r][c][i], sh[q % 2][0][0][i]));
                        uint32_t w[C::WPT];
                        pack_tile<MP>(y, w);
                        store_tile<MP>(w, T0 + r, c, act, C::ACT_STRIDE, lane);
                    });
                    __syncthreads();
                }

                // output layer (5 x H, rows padded to one tile): wave w, sample column tile w
                {
                    f32x16 out[1][1];
                    init_bias<1, 1>(out, make_rsrc(p.bias[kMaxLayers - 1], p.bias_bytes[kMaxLayers - 1]), 0, lane);
                    mma_pass<MP, 1, 1, C::NKBH>(out, make_rsrc(p.wA[kMaxLayers - 1], p.wA_bytes[kMaxLayers - 1]), 0,
                                                act, C::ACT_STRIDE, wave, lane, nohook);
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
        }

        if (tid < kTileM) {
            const int64_t i = base + tid;
            float xk[5];
            if constexpr (rk4 && !fold) {
                advance(nevals - 1, xk);
            } else {
#pragma unroll
                for (int d = 0; d < 5; ++d) xk[d] = xs[d * kTileM + tid];
            }
            if (i < n_items) sampler_outputs(p, i, xk);
        }
        __syncthreads();
    }
}

template <int MP, int H>
hipError_t launch_film(const MlpParams &p, int cu, hipStream_t s)
{
    constexpr int threads = FilmCfg<MP, H>::THREADS;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((p.n + kTileM - 1) / kTileM, cu));
    if (p.integrator == 1) hipLaunchKernelGGL((film_ode_kernel<MP, H, 1>), dim3(grid), dim3(threads), 0, s, p);
    else hipLaunchKernelGGL((film_ode_kernel<MP, H, 0>), dim3(grid), dim3(threads), 0, s, p);
    return hipGetLastError();
}

}  // namespace

bool film_supported(int prec, int hidden)
{
    if (prec == kF32) return hidden == 128;
    if (prec == kBF16) return hidden == 128 || hidden == 256 || hidden == 512;
    return false;
}

hipError_t launch_film_ode(int prec, int hidden, const MlpParams &p, int cu, hipStream_t s)
{
    switch (prec * 1000 + hidden) {
    case kF32 * 1000 + 128: return launch_film<kF32, 128>(p, cu, s);
    case kBF16 * 1000 + 128: return launch_film<kBF16, 128>(p, cu, s);
    case kBF16 * 1000 + 256: return launch_film<kBF16, 256>(p, cu, s);
    case kBF16 * 1000 + 512: return launch_film<kBF16, 512>(p, cu, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gmc
