// Internal interfaces between the C ABI (gmc_api.cpp) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmc {

enum Prec { kF32 = 0, kBF16 = 1, kFP8 = 2 };

// Samples per workgroup tile of the fused MLP/ODE kernel (and the small tiles of launches with
// at most kSmallTileM or kMidTileM samples per compute unit) and waves per workgroup.
constexpr int kTileM = 128;
constexpr int kSmallTileM = 32;
constexpr int kMidTileM = 64;
constexpr int kWaves = 4;

// Operand geometry of one "k-block" for each operand precision: features consumed per
// k-block, bytes one lane holds per 32-row tile and k-block, MFMA instructions per k-block.
//   fp32: v_mfma_f32_32x32x2_f32,    k-block 8 features, 16 B per lane, 4 MFMA
//   bf16: v_mfma_f32_32x32x16_bf16,  k-block 16 features, 16 B per lane, 1 MFMA
//   fp8:  v_mfma_..._32x32x64_f8f6f4 k-block 64 features, 32 B per lane, 1 MFMA
__host__ __device__ constexpr int kb_width(int p) { return p == kF32 ? 8 : (p == kBF16 ? 16 : 64); }
__host__ __device__ constexpr int frag_bytes(int p) { return p == kFP8 ? 32 : 16; }
__host__ __device__ constexpr int elem_bytes(int p) { return p == kF32 ? 4 : (p == kBF16 ? 2 : 1); }

// Operand precision of each of the five layers for a model precision: FP8 models keep the
// first (10 -> H) and last (H -> 5) layers in BF16.
__host__ __device__ constexpr int layer_prec(int model_prec, int layer)
{
    return model_prec == kFP8 ? ((layer == 0 || layer == 4) ? kBF16 : kFP8) : model_prec;
}

// Logical feature stored at physical column p of the LDS activation tile when the producing
// layer wrote it for a consumer of operand precision `p_in`.  The producer's accumulator of
// 32-row tile T gives lane half h the rows 8*(i/4) + 4*h + (i%4), i = 0..15; these land in the
// columns that the consumer's lane half h reads as one contiguous chunk.
__host__ __device__ inline int phys_to_feature(int p_in, int p)
{
    int T, h, i;
    if (p_in == kF32) {
        const int kb = p / 8;
        h = (p % 8) / 4;
        T = kb / 4;
        i = 4 * (kb % 4) + p % 4;
    } else if (p_in == kBF16) {
        const int kb = p / 16;
        h = (p % 16) / 8;
        T = kb / 2;
        i = 8 * (kb % 2) + p % 8;
    } else {
        const int kb = p / 64, w = p % 64;
        h = w / 32;
        T = 2 * kb + (w % 32) / 16;
        i = w % 16;
    }
    return 32 * T + 8 * (i / 4) + 4 * h + (i % 4);
}

// The residual velocity network with adaptive modulation: embedding width, residual blocks,
// features of its input row ([x (5), time features (8), condition (<= 6)], zero-padded) and
// layers (input, embedding, main / scale / shift per block, output).
constexpr int kFilmEmb = 32;
constexpr int kFilmBlocks = 3;
constexpr int kFilmIn = 32;
constexpr int kMaxLayers = 3 + 3 * kFilmBlocks;

struct MlpParams {
    int net;                  // 0: plain MLP (5 layers), 1: residual network (kMaxLayers layers)
    const void *wA[kMaxLayers];     // arranged operand fragments per layer
    const float *bias[kMaxLayers];  // per layer, rows padded to a multiple of 32, pre-divided by oscale
    uint32_t wA_bytes[kMaxLayers], bias_bytes[kMaxLayers];   // sizes (bounds of the buffer loads)
    float oscale[5];          // accumulator multiplier per layer (1 in every model built here)
    float inv_in_scale[5];    // factor of the activation stored as layer l's input: FP8 hidden
                              // layers 1 / (2 sa) (the halved scaled activation over the
                              // layer's activation scale), else 1
    const float *log_tau, *c, *y_in, *sin_th;
    const float *x_in, *cos_phi;   // internal model only: birth x and direction cosine
    const float *log_aspect;  // rectangular boundary model: ln(width / entry-face length), or NULL
    int n_cond;               // condition features: 4 (boundary), 5 (rectangular), 6 (internal)
    const float *noise;       // optional [5][n]
    float *raw;               // optional [5][n]
    const uint64_t *ids;      // optional per-sample random stream ids (else id_base + i)
    const uint64_t *keys;     // optional per-sample Philox keys (else seed)
    int32_t *face;
    float *pos, *dcos, *dsin, *path;
    int64_t n;                // samples (also the row stride of noise / raw)
    const unsigned long long *n_dev;   // optional: sample count read on the device (<= n)
    int K;                    // integration steps
    int integrator;           // 0 explicit Euler, 1 classic RK4 (4 evaluations per step)
    const float *omega_x;     // XY boundary model: in-plane x component of the entry direction
    int xy;                   // XY geometry: exit directions decoded into the unit disk
    uint64_t seed, id_base;
    // Device-side tile choice, for launches whose count n_dev is known only on the device and
    // whose bound n exceeds what 32-sample tiles serve: the launcher runs the smaller-tile
    // kernels first, 32 then 64 samples; each reads its count, and its first lane writes to
    // its n_dev_large the count left to the next kernel (0 when the count is at most its
    // small_max, else the whole count); it exits when that count is not 0, and the next kernel
    // takes that word as its n_dev.  The caller passes two words of device memory (NULL: no
    // device-side choice), one per handoff; the launcher sets each kernel's word and small_max.
    unsigned long long *n_dev_large;
    int64_t small_max;
    // FP8 hidden layers: E8M0 byte (127 + e) of the matrix core's operand scale 2^e = 2 sw sa
    // (weight and activation scales, and the 2 that undoes the halving), else 127
    int32_t mscale[5];
};

// One fused sampler launch over p.n samples (the launch's bound: p.n_dev, when set, holds the
// count) for the network p.net (plain MLP or residual network) on a device of cu compute units:
// the launcher picks the tile size and a grid of at most cu persistent workgroups.
hipError_t launch_mlp_ode(int prec, int hidden, const MlpParams &p, int cu, hipStream_t s);
bool mlp_supported(int prec, int hidden);
// Takes the occupancy query behind the persistent grid of the plain network's kernels at this
// precision and width (outside any stream capture: called when a model is created).
void mlp_prepare(int prec, int hidden);
hipError_t launch_film_ode(int prec, int hidden, const MlpParams &p, int cu, hipStream_t s);
bool film_supported(int prec, int hidden);

struct WalkParams {
    const float *log_tau, *c, *y_in, *sin_th;
    const float *x_in, *cos_phi;   // optional: start inside the cell at (x_in, y_in), direction
                                   // (cos_phi, sin_th); else on the left face, cosine from sin_th
    const float *log_aspect;  // optional: cell [0, A] x [0, 1], A = exp(log_aspect); else square
    const float *omega_x;     // optional: XY geometry, in-plane x component of the entry direction
    int32_t *face;
    float *pos, *dcos, *dsin, *path;
    uint32_t *ncoll;          // optional
    const uint64_t *ids;      // optional per-particle random stream ids (else id_base + i)
    const uint64_t *keys;     // optional per-particle Philox keys (else seed)
    int64_t n;
    const unsigned long long *n_dev;   // optional: particle count read on the device (<= n)
    int mode;
    uint64_t seed, id_base;
    unsigned long long *queue;  // device work counter, zeroed by the launcher
};

hipError_t launch_walk(const WalkParams &p, int grid, hipStream_t s);
#ifndef GMC_WALK_BLOCKS_PER_CU
#define GMC_WALK_BLOCKS_PER_CU 8
#endif
// Grid of the persistent walk for n particles: at most GMC_WALK_BLOCKS_PER_CU blocks of 256
// lanes per compute unit.
inline int walk_grid(int64_t n, int cu)
{
    const int64_t want = (n + 255) / 256, cap = (int64_t)cu * GMC_WALK_BLOCKS_PER_CU;
    return (int)(want < cap ? want : cap);
}
hipError_t launch_split(const WalkParams &p, int32_t *flag, hipStream_t s);
hipError_t launch_decode(const float *raw, int64_t n, int32_t *face, float *pos, float *dcos,
                         float *dsin, float *path, int32_t *flags, hipStream_t s);

int device_cu_count();
// The next work counter of the analog walk's ring on the current device (allocated by
// gmc_device_init), or nullptr if the device has not been set up.
unsigned long long *device_queue_counter();
// Work counters of the allocation-free walk (mc_transmit_noalloc): a file-scope device array of
// kNoAllocCounters counters in gmc_walk.hip.  lookup_noalloc_counters gives its address on the
// current device (a host-side lookup, no allocation).
constexpr int kNoAllocCounters = 64;
hipError_t lookup_noalloc_counters(unsigned long long **base);

// Record a thread-local error message (returned by gmc_last_error) and return `code`.
int set_error(int code, const char *msg);
int set_hip_error(hipError_t e, const char *what);

}  // namespace gmc

struct gmc_model {
    uint64_t serial = 0;     // unique per created model (keys captured launches)
    int precision = 0;
    int hidden = 0;
    int n_in = 10;           // 10: boundary model, 11: rectangular-cell or XY boundary model, 12: internal
    bool xy = false;         // XY geometry (blob flags bit 0): condition carries omega_x
    bool collided = false;   // fitted on collided exits (blob flags bit 1): transport splits first flights
    bool film = false;       // residual network with adaptive modulation (blob flags bit 2)
    int device = 0;
    void *dev_mem = nullptr;
    gmc::MlpParams tmpl{};   // weight / bias pointers and scales
};
