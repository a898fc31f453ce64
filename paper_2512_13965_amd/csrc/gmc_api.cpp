// C ABI of the gfx950 Generative Monte Carlo library: argument checking, error reporting,
// model upload (weights re-arranged into MFMA fragment order) and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gmc.h"
#include "gmc_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(GMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- host-side rounding used when uploading weights -------------------------------------

uint16_t f32_to_bf16_rne(float f)
{
    uint32_t b;
    std::memcpy(&b, &f, 4);
    const uint32_t lsb = (b >> 16) & 1u;
    return (uint16_t)((b + 0x7FFFu + lsb) >> 16);
}

// Value of the OCP e4m3 code c (0..0x7E positive finite codes).
double e4m3_value(int c)
{
    const int e = (c >> 3) & 15, m = c & 7;
    return e == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7);
}

// Nearest e4m3 code, ties to the even code, saturating at 448.
uint8_t f32_to_e4m3_rne_sat(float f)
{
    static std::vector<double> table;
    static std::once_flag once;
    std::call_once(once, [] {
        table.resize(127);
        for (int c = 0; c < 127; ++c) table[c] = e4m3_value(c);
    });
    const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
    const double a = std::fabs((double)f);
    if (a >= 448.0) return sign | 0x7E;
    const auto it = std::upper_bound(table.begin(), table.end(), a);
    const int hi = (int)(it - table.begin());      // first code with value > a
    if (hi == 0) return sign;
    const int lo = hi - 1;
    if (hi >= 127 || table[lo] == a) return sign | (uint8_t)lo;
    const double dl = a - table[lo], dh = table[hi] - a;
    int c = dl < dh ? lo : (dh < dl ? hi : ((lo & 1) == 0 ? lo : hi));
    return sign | (uint8_t)c;
}

struct BlobHeader {
    char magic[8];
    uint32_t version, n_in, hidden, n_out, n_layers, flags, seed, reserved;
    float act_scale[5], w_scale[5];
};
static_assert(sizeof(BlobHeader) == 80, "blob header layout");

bool is_pow2(float s)
{
    if (!(s > 0.0f) || !std::isfinite(s)) return false;
    int e;
    return std::frexp(s, &e) == 0.5f;
}

std::mutex g_dev_mu;
int g_cu[64] = {0};
unsigned long long *g_queue[64] = {nullptr};
unsigned g_queue_next[64] = {0};
constexpr int kQueueRing = 4096;
unsigned long long *g_noalloc[64] = {nullptr};   // address of the allocation-free walk's counters
unsigned g_noalloc_next[64] = {0};
// Largest n of mc_transmit_noalloc: its work counter (64 bits) runs up to n plus one chunk
// per wave.
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 62;


}  // namespace

namespace gmc {

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_cu[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        g_cu[dev] = cu;
    }
    return g_cu[dev];
}

// A ring of per-call work counters on the current device (allocated by gmc_device_init, kept
// until the process ends).  Each launch takes the next slot and zeroes it on its own stream
// first.
unsigned long long *device_queue_counter()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_queue[dev]) return nullptr;
    unsigned slot = g_queue_next[dev]++ % kQueueRing;
    return g_queue[dev] + slot;
}

// The next counter of the allocation-free walk on the current device, or nullptr if the device
// has not been set up.
unsigned long long *noalloc_counter()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_noalloc[dev]) return nullptr;
    unsigned slot = g_noalloc_next[dev]++ % gmc::kNoAllocCounters;
    return g_noalloc[dev] + slot;
}

}  // namespace gmc

namespace gmc {
int set_error(int code, const char *msg) { return fail(code, msg); }
int set_hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }
}  // namespace gmc

extern "C" {

const char *gmc_last_error(void) { return g_err.c_str(); }

int gmc_device_init(void)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "gmc_device_init: hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(GMC_EUNSUPPORTED, "gmc_device_init: device index beyond 63");
    if (gmc::device_cu_count() <= 0) return fail(GMC_EDEVICE, "gmc_device_init: cannot query the device");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_queue[dev]) {
        void *p = nullptr;
        e = hipMalloc(&p, sizeof(unsigned long long) * kQueueRing);
        if (e != hipSuccess) return fail(GMC_ENOMEM, "gmc_device_init: cannot allocate the walk's work counters");
        g_queue[dev] = (unsigned long long *)p;
    }
    if (!g_noalloc[dev]) {     // once per device, with that device current
        unsigned long long *base = nullptr;
        e = gmc::lookup_noalloc_counters(&base);
        if (e != hipSuccess) return hip_fail(e, "gmc_device_init: looking up the allocation-free walk's counters");
        g_noalloc[dev] = base;
    }
    return GMC_OK;
}

int gmc_model_create(const void *host_blob, size_t nbytes, int precision, gmc_model **out)
{
    using namespace gmc;
    if (!host_blob || !out) return fail(GMC_EINVAL, "gmc_model_create: null pointer");
    *out = nullptr;
    if (precision < GMC_FP32 || precision > GMC_FP8_E4M3)
        return fail(GMC_EINVAL, "gmc_model_create: unknown precision");
    if (nbytes < sizeof(BlobHeader)) return fail(GMC_EINVAL, "gmc_model_create: blob too small");
    BlobHeader hd;
    std::memcpy(&hd, host_blob, sizeof hd);
    if (std::memcmp(hd.magic, "GMCW0001", 8) != 0 || hd.version != 1)
        return fail(GMC_EINVAL, "gmc_model_create: bad magic or version");
    const bool film = (hd.flags & 4u) != 0;
    if (hd.n_in < 10 || hd.n_in > 12 || hd.n_out != 5)
        return fail(GMC_EINVAL, "gmc_model_create: network must have 10, 11 or 12 inputs and 5 outputs");
    if (!film && hd.n_layers != 5)
        return fail(GMC_EINVAL, "gmc_model_create: the plain network is 10, 11 or 12 -> H x4 -> 5");
    if (film && (hd.n_layers != (uint32_t)kFilmBlocks || hd.reserved != (uint32_t)kFilmEmb))
        return fail(GMC_EINVAL, "gmc_model_create: the residual network has " + std::to_string(kFilmBlocks) +
                                    " blocks and embedding width " + std::to_string(kFilmEmb));
    if (hd.flags & ~7u) return fail(GMC_EINVAL, "gmc_model_create: unknown flags");
    if ((hd.flags & 2u) && hd.n_in == 12)
        return fail(GMC_EINVAL, "gmc_model_create: only boundary models can be fitted on collided exits");
    if ((hd.flags & 1u) && hd.n_in != 11)
        return fail(GMC_EINVAL, "gmc_model_create: an XY-geometry model has 11 inputs");
    const int H = (int)hd.hidden;
    if (film ? !film_supported(precision, H) : !mlp_supported(precision, H))
        return fail(GMC_EUNSUPPORTED, std::string("gmc_model_create: ") + (film ? "residual network" : "network") +
                                          " of hidden width " + std::to_string(H) +
                                          " not built for this precision");
    const int NI = (int)hd.n_in, NC = NI - 6;
    // [out, in] of every layer in blob order: the plain MLP's five layers, or the residual
    // network's input layer [x, time features, condition], embedding [time features,
    // condition], (main, scale, shift) per block and output layer
    std::vector<std::array<int, 2>> dims;
    if (film) {
        dims.push_back({H, 13 + NC});
        dims.push_back({kFilmEmb, 8 + NC});
        for (int j = 0; j < kFilmBlocks; ++j) {
            dims.push_back({H, H});
            dims.push_back({H, kFilmEmb});
            dims.push_back({H, kFilmEmb});
        }
        dims.push_back({5, H});
    } else {
        dims = {{H, NI}, {H, H}, {H, H}, {H, H}, {5, H}};
    }
    const int NL = (int)dims.size();
    size_t need = sizeof(BlobHeader);
    for (auto &d : dims) need += sizeof(float) * (size_t)(d[0] * d[1] + d[0]);
    if (nbytes != need) return fail(GMC_EINVAL, "gmc_model_create: blob size does not match header");
    for (int l = 0; l < 5; ++l)
        if (!is_pow2(hd.act_scale[l]) || !is_pow2(hd.w_scale[l]))
            return fail(GMC_EINVAL, "gmc_model_create: scales must be positive powers of two");
    // FP8 layers apply 2 w_scale act_scale as the matrix core's E8M0 operand scale
    if (precision == GMC_FP8_E4M3 && !film)
        for (int l = 0; l < 5; ++l) {
            if (layer_prec(precision, l) != kFP8) continue;
            const double e = std::log2(2.0 * (double)hd.w_scale[l] * (double)hd.act_scale[l]);
            if (e < -127.0 || e > 127.0)
                return fail(GMC_EINVAL, "gmc_model_create: FP8 layer scales out of the E8M0 range");
        }

    const float *src = (const float *)((const char *)host_blob + sizeof(BlobHeader));
    std::vector<const float *> W(NL), B(NL);
    for (int l = 0; l < NL; ++l) {
        W[l] = src;
        src += dims[l][0] * dims[l][1];
        B[l] = src;
        src += dims[l][0];
        for (int i = 0; i < dims[l][0] * (dims[l][1] + 1); ++i)
            if (!std::isfinite(W[l][i])) return fail(GMC_EINVAL, "gmc_model_create: non-finite weight");
    }

    const int irc = gmc_device_init();     // the blob is valid: set up the device
    if (irc != GMC_OK) return irc;

    // arrange every layer into fragment order, then one device allocation for all of it
    std::vector<std::vector<uint8_t>> frag(NL);
    std::vector<std::vector<float>> bias(NL);
    gmc_model *m = new gmc_model();
    static std::atomic<uint64_t> next_serial{1};
    m->serial = next_serial++;
    m->precision = precision;
    m->n_in = NI;
    m->xy = (hd.flags & 1u) != 0;
    m->collided = (hd.flags & 2u) != 0;
    m->film = film;
    m->tmpl.net = film ? 1 : 0;
    m->tmpl.xy = m->xy ? 1 : 0;
    m->tmpl.n_cond = NC;
    m->hidden = H;
    // BF16 and FP8 plain networks carry their hidden activations scaled by -log2(e) (the
    // sampler's SiLU then takes its exponential without a multiply): the first layer's weights
    // and every hidden bias times -log2(e), the output layer's weights times -ln 2, each
    // product rounded to float32 before the BF16 rounding of the weights.  The e4m3 hidden
    // layers keep their weights; they take half the scaled activation over their activation
    // scale sa (the same headroom below e4m3's 448 as the plain SiLU) and multiply their sum by
    // 2 sw sa on the matrix core (its E8M0 operand scale), so their accumulators hold the
    // scaled pre-activation with the bias added unscaled.
    const bool fold = !film && (precision == GMC_BF16 || precision == GMC_FP8_E4M3);
    constexpr float kNegLog2e = -1.4426950408889634f, kNegLn2 = -0.6931471805599453f;
    auto weight_factor = [&](int l) { return !fold ? 1.0f : (l == 0 ? kNegLog2e : (l == NL - 1 ? kNegLn2 : 1.0f)); };
    auto bias_factor = [&](int l) { return (fold && l < NL - 1) ? kNegLog2e : 1.0f; };
    for (int l = 0; l < NL; ++l) {
        const int P = film ? precision : layer_prec(precision, l);
        const int KBW = kb_width(P), FB = frag_bytes(P), EB = elem_bytes(P);
        const int out_dim = dims[l][0], in_dim = dims[l][1];
        // padded input width and the blob column of physical input column k (-1: zero).  The
        // first layers read rows the threads wrote in natural order: the plain input
        // [x, t, condition]; the residual network's [x (0..4), time features (5..12),
        // condition (13..)], of which its embedding reads columns 5 on.  Every other layer
        // reads a tile its producer's accumulators stored (phys_to_feature).
        const bool first = (l == 0) || (film && l == 1);
        const bool from_emb = film && l >= 2 && l < NL - 1 && (l - 2) % 3 != 0;
        const int kpad = first ? (film ? kFilmIn : 16) : (from_emb ? kFilmEmb : H);
        auto column = [&](int k) {
            if (!first) return phys_to_feature(P, k);
            if (film && l == 1) return k >= 5 ? k - 5 : -1;
            return k;
        };
        const int nkb = kpad / KBW, nt = (out_dim + 31) / 32;
        const bool f8 = (P == kFP8);
        const float sw = f8 ? hd.w_scale[l] : 1.0f, sa = f8 ? hd.act_scale[l] : 1.0f;
        if (l < 5) {
            m->tmpl.oscale[l] = 1.0f;
            m->tmpl.inv_in_scale[l] = f8 ? 0.5f / sa : 1.0f;
            m->tmpl.mscale[l] = 127;
            if (f8) m->tmpl.mscale[l] = 127 + (int)std::lround(std::log2(2.0 * (double)sw * (double)sa));
        }
        frag[l].assign((size_t)nt * nkb * 64 * FB, 0);
        for (int T = 0; T < nt; ++T)
            for (int kb = 0; kb < nkb; ++kb)
                for (int lane = 0; lane < 64; ++lane) {
                    const int row = 32 * T + (lane & 31), h = lane >> 5;
                    uint8_t *dst = frag[l].data() + ((size_t)(T * nkb + kb) * 64 + lane) * FB;
                    for (int e = 0; e < KBW / 2; ++e) {
                        const int k = kb * KBW + h * (KBW / 2) + e;
                        const int f = column(k);
                        const float w = (row < out_dim && f >= 0 && f < in_dim)
                                            ? W[l][(size_t)row * in_dim + f] * weight_factor(l) : 0.0f;
                        if (P == kF32) {
                            std::memcpy(dst + e * EB, &w, 4);
                        } else if (P == kBF16) {
                            const uint16_t q = f32_to_bf16_rne(w);
                            std::memcpy(dst + e * EB, &q, 2);
                        } else {
                            dst[e] = f32_to_e4m3_rne_sat(w / sw);
                        }
                    }
                }
        // the residual network's scale maps carry the "1 +" of the modulation in their bias
        const float one = (film && l >= 2 && l < NL - 1 && (l - 2) % 3 == 1) ? 1.0f : 0.0f;
        bias[l].assign((size_t)nt * 32, 0.0f);
        for (int r = 0; r < out_dim; ++r) bias[l][r] = B[l][r] * bias_factor(l) + one;
    }
    static_assert(3 + 3 * kFilmBlocks == kMaxLayers, "the residual network fills every layer slot");
    size_t total = 0;
    std::vector<size_t> off_f(NL), off_b(NL);
    for (int l = 0; l < NL; ++l) {
        off_f[l] = total;
        total += (frag[l].size() + 255) & ~(size_t)255;
        off_b[l] = total;
        total += (bias[l].size() * sizeof(float) + 255) & ~(size_t)255;
    }
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) { delete m; return hip_fail(e, "gmc_model_create: hipGetDevice"); }
    e = hipMalloc(&m->dev_mem, total);
    if (e != hipSuccess) { delete m; return fail(GMC_ENOMEM, "gmc_model_create: hipMalloc failed"); }
    std::vector<uint8_t> staging(total, 0);
    for (int l = 0; l < NL; ++l) {
        std::memcpy(staging.data() + off_f[l], frag[l].data(), frag[l].size());
        std::memcpy(staging.data() + off_b[l], bias[l].data(), bias[l].size() * sizeof(float));
        m->tmpl.wA[l] = (const char *)m->dev_mem + off_f[l];
        m->tmpl.bias[l] = (const float *)((const char *)m->dev_mem + off_b[l]);
        m->tmpl.wA_bytes[l] = (uint32_t)frag[l].size();
        m->tmpl.bias_bytes[l] = (uint32_t)(bias[l].size() * sizeof(float));
    }
    e = hipMemcpy(m->dev_mem, staging.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(m->dev_mem);
        delete m;
        return hip_fail(e, "gmc_model_create: upload");
    }
    if (!film) mlp_prepare(precision, H);
    *out = m;
    return GMC_OK;
}

int gmc_model_destroy(gmc_model *m)
{
    if (!m) return fail(GMC_EINVAL, "gmc_model_destroy: null model");
    if (m->dev_mem) {
        hipError_t e = hipFree(m->dev_mem);
        if (e != hipSuccess) { delete m; return hip_fail(e, "gmc_model_destroy"); }
    }
    delete m;
    return GMC_OK;
}

int gmc_model_info(const gmc_model *m, int *hidden, int *precision)
{
    if (!m) return fail(GMC_EINVAL, "gmc_model_info: null model");
    if (hidden) *hidden = m->hidden;
    if (precision) *precision = m->precision;
    return GMC_OK;
}

int gmc_model_inputs(const gmc_model *m, int *n_in)
{
    if (!m || !n_in) return fail(GMC_EINVAL, "gmc_model_inputs: null pointer");
    *n_in = m->n_in;
    return GMC_OK;
}

static bool cond_ok(const gmc_cond &c) { return c.log_tau && c.c && c.y_in && c.sin_th; }
static bool cond_ok(const gmc_cond_internal &c)
{
    return c.log_tau && c.c && c.x && c.y && c.cos_phi && c.sin_phi;
}
static bool exit_ok(const gmc_exit &o) { return o.face && o.pos && o.dir_cos && o.dir_sin && o.path; }

int gmc_transmit(const gmc_model *m, gmc_cond cond, int64_t n, int K, uint64_t seed,
                 uint64_t id_base, const float *noise_opt, float *raw_opt, gmc_exit out, void *stream)
{
    return gmc_sample(m, cond, n, GMC_EULER, K, seed, id_base, noise_opt, raw_opt, out, stream);
}

}  // extern "C"

namespace {

// Common part of gmc_sample / gmc_sample_internal: checks, then one fused sampler launch with the
// condition pointers already in p.
int launch_sampler(const gmc_model *m, gmc::MlpParams p, int64_t n, int integrator, int K, uint64_t seed,
                   uint64_t id_base, const float *noise_opt, float *raw_opt, gmc_exit out, void *stream,
                   const char *who)
{
    const std::string w(who);
    if (integrator != GMC_EULER && integrator != GMC_RK4)
        return fail(GMC_EINVAL, w + ": integrator must be GMC_EULER or GMC_RK4");
    if (K < 1 || K > 1024) return fail(GMC_EINVAL, w + ": K must be in 1..1024");
    if (n == 0) return GMC_OK;
    if (!exit_ok(out)) return fail(GMC_EINVAL, w + ": null output array");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device)
        return fail(GMC_EINVAL, w + ": model lives on another device");
    p.noise = noise_opt;
    p.raw = raw_opt;
    p.face = out.face;
    p.pos = out.pos;
    p.dcos = out.dir_cos;
    p.dsin = out.dir_sin;
    p.path = out.path;
    p.n = n;
    p.n_dev = nullptr;
    p.K = K;
    p.integrator = integrator;
    p.seed = seed;
    p.id_base = id_base;
    const int cu = gmc::device_cu_count();
    if (cu <= 0) return fail(GMC_EDEVICE, w + ": cannot query the device");
    hipError_t e = gmc::launch_mlp_ode(m->precision, m->hidden, p, cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, (w + ": launch").c_str());
    return GMC_OK;
}

int launch_walk_api(gmc::WalkParams p, int64_t n, int mode, uint64_t seed, uint64_t id_base, gmc_exit out,
                    uint32_t *ncoll_opt, void *stream, const char *who, bool noalloc = false)
{
    const std::string w(who);
    if (mode != GMC_MODE_CONTINUOUS && mode != GMC_MODE_ANALOG)
        return fail(GMC_EINVAL, w + ": mode must be 0 (continuous) or 1 (analog)");
    if (n == 0) return GMC_OK;
    if (!exit_ok(out)) return fail(GMC_EINVAL, w + ": null output array");
    p.face = out.face;
    p.pos = out.pos;
    p.dcos = out.dir_cos;
    p.dsin = out.dir_sin;
    p.path = out.path;
    p.ncoll = ncoll_opt;
    p.n = n;
    p.n_dev = nullptr;
    p.mode = mode;
    p.seed = seed;
    p.id_base = id_base;
    p.queue = noalloc ? gmc::noalloc_counter() : gmc::device_queue_counter();
    if (!p.queue) return fail(GMC_EINVAL, w + ": gmc_device_init has not been called on this device");
    const int cu = gmc::device_cu_count();
    if (cu <= 0) return fail(GMC_EDEVICE, w + ": cannot query the device");
    const int grid = gmc::walk_grid(n, cu);
    hipError_t e = gmc::launch_walk(p, grid, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, (w + ": launch").c_str());
    return GMC_OK;
}

}  // namespace

extern "C" {

int gmc_sample(const gmc_model *m, gmc_cond cond, int64_t n, int integrator, int K, uint64_t seed,
               uint64_t id_base, const float *noise_opt, float *raw_opt, gmc_exit out, void *stream)
{
    if (!m) return fail(GMC_EINVAL, "gmc_transmit: null model");
    if (n < 0) return fail(GMC_EINVAL, "gmc_transmit: negative n");
    if (m->n_in != 10 && m->n_in != 11)
        return fail(GMC_EINVAL, "gmc_transmit: the model is not a boundary model (10 or 11 inputs)");
    if (m->n_in == 10 && cond.log_aspect)
        return fail(GMC_EINVAL, "gmc_transmit: a square-cell model (10 inputs) takes no aspect ratio");
    if ((cond.omega_x != nullptr) != m->xy)
        return fail(GMC_EINVAL, "gmc_transmit: omega_x is given exactly for XY-geometry models");
    if (m->xy && cond.log_aspect)
        return fail(GMC_EINVAL, "gmc_transmit: XY-geometry models serve square cells");
    if (n > 0 && !cond_ok(cond)) return fail(GMC_EINVAL, "gmc_transmit: null condition array");
    gmc::MlpParams p = m->tmpl;
    p.log_tau = cond.log_tau;
    p.c = cond.c;
    p.y_in = cond.y_in;
    p.sin_th = cond.sin_th;
    p.x_in = nullptr;
    p.cos_phi = nullptr;
    p.log_aspect = cond.log_aspect;
    p.omega_x = cond.omega_x;
    return launch_sampler(m, p, n, integrator, K, seed, id_base, noise_opt, raw_opt, out, stream, "gmc_sample");
}

int gmc_sample_internal(const gmc_model *m, gmc_cond_internal cond, int64_t n, int integrator, int K,
                        uint64_t seed, uint64_t id_base, const float *noise_opt, float *raw_opt,
                        gmc_exit out, void *stream)
{
    if (!m) return fail(GMC_EINVAL, "gmc_sample_internal: null model");
    if (n < 0) return fail(GMC_EINVAL, "gmc_sample_internal: negative n");
    if (m->n_in != 12) return fail(GMC_EINVAL, "gmc_sample_internal: the model is not an internal model (12 inputs)");
    if (n > 0 && !cond_ok(cond)) return fail(GMC_EINVAL, "gmc_sample_internal: null condition array");
    gmc::MlpParams p = m->tmpl;
    p.log_tau = cond.log_tau;
    p.c = cond.c;
    p.x_in = cond.x;
    p.y_in = cond.y;
    p.cos_phi = cond.cos_phi;
    p.sin_th = cond.sin_phi;
    return launch_sampler(m, p, n, integrator, K, seed, id_base, noise_opt, raw_opt, out, stream,
                          "gmc_sample_internal");
}

int mc_transmit(gmc_cond cond, int64_t n, int mode, uint64_t seed, uint64_t id_base, gmc_exit out,
                uint32_t *ncoll_opt, void *stream)
{
    if (n < 0) return fail(GMC_EINVAL, "mc_transmit: negative n");
    if (n > 0 && !cond_ok(cond)) return fail(GMC_EINVAL, "mc_transmit: null condition array");
    gmc::WalkParams p{};
    p.log_tau = cond.log_tau;
    p.c = cond.c;
    p.y_in = cond.y_in;
    p.sin_th = cond.sin_th;
    p.log_aspect = cond.log_aspect;
    p.omega_x = cond.omega_x;
    return launch_walk_api(p, n, mode, seed, id_base, out, ncoll_opt, stream, "mc_transmit");
}

int mc_transmit_noalloc(gmc_cond cond, int64_t n, int mode, uint64_t seed, uint64_t id_base, gmc_exit out,
                        uint32_t *ncoll_opt, void *stream)
{
    if (n < 0) return fail(GMC_EINVAL, "mc_transmit_noalloc: negative n");
    if (n > kNoAllocMaxN)
        return fail(GMC_EINVAL, "mc_transmit_noalloc: n beyond 2^62, the range of its work counter");
    if (n > 0 && !cond_ok(cond)) return fail(GMC_EINVAL, "mc_transmit_noalloc: null condition array");
    gmc::WalkParams p{};
    p.log_tau = cond.log_tau;
    p.c = cond.c;
    p.y_in = cond.y_in;
    p.sin_th = cond.sin_th;
    p.log_aspect = cond.log_aspect;
    p.omega_x = cond.omega_x;
    return launch_walk_api(p, n, mode, seed, id_base, out, ncoll_opt, stream, "mc_transmit_noalloc", true);
}

int mc_transmit_internal(gmc_cond_internal cond, int64_t n, int mode, uint64_t seed, uint64_t id_base,
                         gmc_exit out, uint32_t *ncoll_opt, void *stream)
{
    if (n < 0) return fail(GMC_EINVAL, "mc_transmit_internal: negative n");
    if (n > 0 && !cond_ok(cond)) return fail(GMC_EINVAL, "mc_transmit_internal: null condition array");
    gmc::WalkParams p{};
    p.log_tau = cond.log_tau;
    p.c = cond.c;
    p.x_in = cond.x;
    p.y_in = cond.y;
    p.cos_phi = cond.cos_phi;
    p.sin_th = cond.sin_phi;
    return launch_walk_api(p, n, mode, seed, id_base, out, ncoll_opt, stream, "mc_transmit_internal");
}

int gmc_uncollided_split(gmc_cond cond, int64_t n, uint64_t seed, uint64_t id_base, int32_t *uncollided,
                         gmc_exit out, void *stream)
{
    if (n < 0) return fail(GMC_EINVAL, "gmc_uncollided_split: negative n");
    if (n == 0) return GMC_OK;
    if (!cond_ok(cond) || !uncollided || !exit_ok(out))
        return fail(GMC_EINVAL, "gmc_uncollided_split: null pointer");
    if (n > (int64_t)0x7FFFFFFF * 256) return fail(GMC_EINVAL, "gmc_uncollided_split: n too large");
    gmc::WalkParams p{};
    p.log_tau = cond.log_tau;
    p.c = cond.c;
    p.y_in = cond.y_in;
    p.sin_th = cond.sin_th;
    p.log_aspect = cond.log_aspect;
    p.omega_x = cond.omega_x;
    p.face = out.face;
    p.pos = out.pos;
    p.dcos = out.dir_cos;
    p.dsin = out.dir_sin;
    p.path = out.path;
    p.n = n;
    p.seed = seed;
    p.id_base = id_base;
    hipError_t e = gmc::launch_split(p, uncollided, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gmc_uncollided_split: launch");
    return GMC_OK;
}

int gmc_decode(const float *raw, int64_t n, gmc_exit out, int32_t *flags_opt, void *stream)
{
    if (n < 0) return fail(GMC_EINVAL, "gmc_decode: negative n");
    if (n == 0) return GMC_OK;
    if (!raw || !exit_ok(out)) return fail(GMC_EINVAL, "gmc_decode: null pointer");
    if (n > (int64_t)0x7FFFFFFF * 256) return fail(GMC_EINVAL, "gmc_decode: n too large");
    hipError_t e = gmc::launch_decode(raw, n, out.face, out.pos, out.dir_cos, out.dir_sin, out.path,
                                      flags_opt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gmc_decode: launch");
    return GMC_OK;
}

}  // extern "C"
