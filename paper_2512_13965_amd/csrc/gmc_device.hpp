// Device-side helpers shared by the gfx950 kernels: counter-based random numbers, uniform and
// normal variates, fast transcendentals, and the exit-record decoder.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmc {

constexpr uint32_t kTagNoise = 1u;
constexpr uint32_t kTagWalk = 2u;
constexpr uint32_t kTagSource = 3u;
constexpr uint32_t kTagSplit = 4u;
constexpr uint32_t kMaxFlights = 1u << 24;

struct U4 {
    uint32_t a, b, c, d;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32 -> 64 bit
// multiplies with a Weyl key schedule.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64 bit multiply per product (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw4(uint64_t seed, uint64_t stream, uint32_t index, uint32_t tag)
{
    return philox((uint32_t)stream, (uint32_t)(stream >> 32), index, tag, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// xi in (0, 1]: the top 24 bits plus one ulp, exact in float32.
__device__ __forceinline__ float u01(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1p-24f; }
__device__ __forceinline__ float u01_open(uint32_t w) { return ((float)(w >> 8) + 0.5f) * 0x1p-24f; }

// -ln(xi) from the hardware base-2 logarithm.
__device__ __forceinline__ float neg_log(float xi) { return -0.69314718055994531f * __builtin_amdgcn_logf(xi); }

// cos / sin of 2 pi x: the hardware sine and cosine take their argument in turns.
__device__ __forceinline__ float cos_turns(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float sin_turns(float x) { return __builtin_amdgcn_sinf(x); }

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// SiLU(a) = a / (1 + e^-a) with the hardware exp2 and reciprocal.
__device__ __forceinline__ float silu(float a)
{
    return a * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * a));
}

// z ~ N(0, I_5) of one particle: Philox words of counters (id, 0, tag) and (id, 1, tag),
// Box-Muller on the pairs (w0,w1), (w2,w3), (w4,w5); accurate library log/sincos (this runs
// once per sample, not in a hot loop).
__device__ __forceinline__ void normal5(uint64_t seed, uint64_t id, float z[5])
{
    const U4 a = draw4(seed, id, 0u, kTagNoise);
    const U4 b = draw4(seed, id, 1u, kTagNoise);
    const uint32_t w[6] = {a.a, a.b, a.c, a.d, b.a, b.b};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const float r = sqrtf(-2.0f * logf(u01(w[2 * p])));
        float s, c;
        sincospif(2.0f * u01(w[2 * p + 1]), &s, &c);
        z[2 * p] = r * c;
        if (2 * p + 1 < 5) z[2 * p + 1] = r * s;
    }
}

// State of one analog walk inside the unit cell (paper section "Monte Carlo Method", eq. 4),
// advanced one flight at a time so a persistent kernel can refill lanes between flights.
struct Walker {
    float x, y, u, v, len, inv_sig, cs;
    float wa;                            // cell width in units of its height (1: square)
    bool xy;                             // XY geometry: (u, v) projects a direction on the sphere
    uint32_t flight, ncoll;
    bool scatter, analog;
};

// mode 0 (continuous absorption): flights ~ Exp(c tau); mode 1 (analog): flights ~ Exp(tau)
// and a collision absorbs when xi > c.  Start at (x, y) with direction (u, v) in the cell
// [0, wa] x [0, 1]; lengths and tau are in units of the cell height.
__device__ __forceinline__ void walker_init(Walker &w, float tau, float c, int mode, float x, float y,
                                            float u, float v, float wa = 1.0f, bool xy = false)
{
    w.wa = wa;
    w.xy = xy;
    w.analog = (mode == 1);
    const float sig = w.analog ? tau : c * tau;
    w.scatter = sig > 1e-30f;            // below this 1/sig would overflow
    w.inv_sig = w.scatter ? 1.0f / sig : 0.0f;
    w.cs = c;
    w.x = x;
    w.y = y;
    w.u = u;
    w.v = v;
    w.len = 0.0f;
    w.flight = 0;
    w.ncoll = 0;
}

constexpr int kInside = -3;

// One flight: distance to the boundary, sampled flight length, then scatter or leave.
// Flight j draws Philox(key, counter (stream lo, stream hi, j, walk tag)): word 0 -> length,
// word 1 -> new direction, word 2 -> absorption test.  Returns kInside while the particle is
// still in the cell, else the exit face 0..3 (pos = counter-clockwise position along it, as a
// fraction of that face's length), -1 absorbed, -2 capped.
__device__ __forceinline__ int walker_flight(Walker &w, uint64_t key, uint64_t stream, float &pos)
{
    const float kInf = __builtin_inff();
    float tx = kInf, ty = kInf;
    if (w.u > 0.0f) tx = (w.wa - w.x) * fast_rcp(w.u);
    else if (w.u < 0.0f) tx = -w.x * fast_rcp(w.u);
    if (w.v > 0.0f) ty = (1.0f - w.y) * fast_rcp(w.v);
    else if (w.v < 0.0f) ty = -w.y * fast_rcp(w.v);
    const bool xface = tx <= ty;
    const float db = fmaxf(xface ? tx : ty, 0.0f);
    const U4 r = draw4(key, stream, w.flight, kTagWalk);
    const float ds = w.scatter ? neg_log(u01(r.a)) * w.inv_sig : kInf;
    int face = kInside;
    if (ds >= db) {
        w.len += db;
        if (xface) {
            const float ye = fminf(fmaxf(w.y + db * w.v, 0.0f), 1.0f);
            face = w.u > 0.0f ? 1 : 3;
            pos = w.u > 0.0f ? ye : 1.0f - ye;
        } else {
            const float xe = fminf(fmaxf(w.x + db * w.u, 0.0f), w.wa);
            face = w.v > 0.0f ? 2 : 0;
            pos = w.v > 0.0f ? (w.wa - xe) / w.wa : xe / w.wa;
        }
    } else {
        w.x += ds * w.u;
        w.y += ds * w.v;
        w.len += ds;
        w.ncoll += 1;
        if (w.analog && u01(r.c) > w.cs) {
            face = -1;
        } else {
            const float ph = u01(r.b);
            w.u = cos_turns(ph);
            w.v = sin_turns(ph);
            if (w.xy) {                  // on the sphere: mu = 2 xi - 1 from word 3, projected
                const float mu = 2.0f * u01(r.d) - 1.0f;
                const float st = sqrtf(fmaxf(1.0f - mu * mu, 0.0f));
                w.u *= st;
                w.v *= st;
            }
        }
    }
    w.flight += 1;
    if (face == kInside && w.flight >= kMaxFlights) face = -2;
    if (face < 0 && face != kInside) pos = 0.0f;
    return face;
}

// Rotation of a direction by k quarter turns counter-clockwise.
__device__ __forceinline__ void rot_quarter(int k, float a, float b, float &ra, float &rb)
{
    switch (k & 3) {
    case 0: ra = a; rb = b; break;
    case 1: ra = -b; rb = a; break;
    case 2: ra = -a; rb = -b; break;
    default: ra = b; rb = -a; break;
    }
}

// Exit record from x_K (paper eq. 11 in the 5-dim reading): face = number of the thresholds
// -1, 0, 1 reached by a4; pos = clamp((a0 + 1) / 2); direction (a1, a2) normalised, outward
// normal if its norm is below 1e-6, normal component reflected if it points inward;
// path = exp(a3).  Returns flags: bit0 pos clamped, bit1 reflected, bit2 zero norm.
struct Exit {
    int32_t face;
    float pos, u, v, path;
};

// In XY geometry the exit direction is a projection: (a1, a2) is kept inside the unit disk
// (scaled to norm 1 only when it lies outside) instead of being normalised.
// Largest |x_d| of a decodable network state: the targets lie within |a| <= 16 (ln path of the
// shortest tracks); a state beyond 32, or not finite, left the fitted range (a rare diverging
// trajectory from the noise's far tail) and is rejected.
constexpr float kDecodeMax = 32.0f;

__device__ __forceinline__ int decode_exit(float a0, float a1, float a2, float a3, float a4, Exit &e,
                                           bool xy = false)
{
    const float amax = fmaxf(fmaxf(fmaxf(fabsf(a0), fabsf(a1)), fmaxf(fabsf(a2), fabsf(a3))), fabsf(a4));
    const bool finite = (a0 - a0 == 0.0f) && (a1 - a1 == 0.0f) && (a2 - a2 == 0.0f) && (a3 - a3 == 0.0f) &&
                        (a4 - a4 == 0.0f);
    if (!finite || !(amax <= kDecodeMax)) {
        e.face = -1;
        e.pos = 0.0f;
        e.u = 0.0f;
        e.v = 0.0f;
        e.path = 0.0f;
        return 8;
    }
    int flags = 0;
    const int face = (a4 >= -1.0f) + (a4 >= 0.0f) + (a4 >= 1.0f);
    float p = (a0 + 1.0f) * 0.5f;
    if (p < 0.0f || p > 1.0f) flags |= 1;
    p = fminf(fmaxf(p, 0.0f), 1.0f);
    // outward normals: bottom (0,-1), right (1,0), top (0,1), left (-1,0)
    const float nx = (face == 1) ? 1.0f : ((face == 3) ? -1.0f : 0.0f);
    const float ny = (face == 2) ? 1.0f : ((face == 0) ? -1.0f : 0.0f);
    const float nrm = sqrtf(a1 * a1 + a2 * a2);
    float u, v;
    if (nrm < 1e-6f) {
        u = nx;
        v = ny;
        flags |= 4;
    } else if (!xy || nrm > 1.0f) {
        const float inv = 1.0f / nrm;
        u = a1 * inv;
        v = a2 * inv;
    } else {
        u = a1;
        v = a2;
    }
    const float dn = u * nx + v * ny;
    if (dn < 0.0f) {
        u -= 2.0f * dn * nx;
        v -= 2.0f * dn * ny;
        flags |= 2;
    }
    e.face = face;
    e.pos = p;
    e.u = u;
    e.v = v;
    e.path = expf(a3);
    return flags;
}

// First-flight split of a canonical transmission: the entry ray from (0, y) along (u, v) meets
// the boundary of [0, wa] x [0, 1] after d_b; with flights ~ Exp(c tau) (eq. 4, continuous
// absorption) the particle crosses without a collision with probability exp(-c tau d_b).  The
// decision compares that probability with xi = u01(word 0) of Philox(key, (id lo, id hi, 0,
// split tag)); an uncollided particle leaves at the ray's end with its entry direction and path
// d_b (written to e).  Returns true for an uncollided crossing.
__device__ __forceinline__ bool uncollided_exit(float tau, float c, float y, float u, float v, float wa,
                                                uint64_t key, uint64_t id, Exit &e)
{
    const float kInf = __builtin_inff();
    const float tx = u > 0.0f ? wa / u : kInf;
    float ty = kInf;
    if (v > 0.0f) ty = (1.0f - y) / v;
    else if (v < 0.0f) ty = -y / v;
    const bool xface = tx <= ty;
    const float db = xface ? tx : ty;
    const float pu = expf(-c * tau * db);
    const U4 r = draw4(key, id, 0u, kTagSplit);
    if (!(u01(r.a) <= pu)) return false;
    e.u = u;
    e.v = v;
    e.path = db;
    if (xface) {
        e.face = 1;
        e.pos = fminf(fmaxf(y + db * v, 0.0f), 1.0f);
    } else {
        const float xe = fminf(fmaxf(db * u, 0.0f), wa);
        e.face = v > 0.0f ? 2 : 0;
        e.pos = v > 0.0f ? (wa - xe) / wa : xe / wa;
    }
    return true;
}

}  // namespace gmc
