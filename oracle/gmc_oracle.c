/*
 * gmc_oracle.c -- plain, slow, FP64 CPU oracle for Generative Monte Carlo cell transmission.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header or table with the GPU path.
 *
 * What it computes (paper: Farmer, Murray, Krotz, McClarren, "Generative Monte Carlo
 * Sampling for Constant-Cost Particle Transport", arXiv 2512.13965):
 *   - analog random walk through one square cell, flights drawn from the scattering
 *     cross section (section "Monte Carlo Method", eq. 4), isotropic flatland scattering,
 *     either with continuous absorption (implicit capture, eqs. 5-6) or with analog
 *     absorption at collisions;
 *   - cell-to-cell transport over a grid with the track-length flux estimator
 *     (eqs. 5-7) and the four stages of section "Transport Algorithm";
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) from its published definition, and
 *     Box-Muller normals, for the counter-based random numbers both sides draw.
 *
 * Conventions (readings of the paper, stated once here):
 *   - unit square [0,1]^2 in units of the cell side L; canonical entry on the left face x=0;
 *   - faces 0 bottom (y=0), 1 right (x=1), 2 top (y=1), 3 left (x=0); the position along an
 *     exit face runs counter-clockwise: bottom x, right y, top 1-x, left 1-y;
 *   - a uniform variate from a 32-bit word u is ((u >> 8) + 1) * 2^-24, in (0, 1];
 *   - corner ties between the x- and y-face go to the x-face.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TAG_NOISE 1u
#define ORC_TAG_WALK 2u
#define ORC_TAG_SOURCE 3u
#define ORC_TAG_SPLIT 4u
#define ORC_MAX_FLIGHTS 16777216u /* 2^24: a walk still inside after this many flights is "capped" */

#define ORC_FACE_ABSORBED (-1)
#define ORC_FACE_CAPPED (-2)

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies, with the */
/* Weyl key schedule between rounds.                                                     */
/* ------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(uint64_t seed, uint64_t stream, uint32_t index, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)stream, (uint32_t)(stream >> 32), index, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* uniform in (0, 1]: the paper's xi of eq. 4 must never be 0 */
double orc_u01(uint32_t u) { return ((double)(u >> 8) + 1.0) * (1.0 / 16777216.0); }

/* uniform in the open interval (0, 1), used for birth positions */
static double u01_open(uint32_t u) { return ((double)(u >> 8) + 0.5) * (1.0 / 16777216.0); }

static const double ORC_PI = 3.14159265358979323846;

/* z ~ N(0, I_5) for one sample (paper eq. 8: the ODE starts from Gaussian noise).
 * Two Philox calls, index 0 and 1 under the noise tag; Box-Muller on the word pairs
 * (w0,w1) -> z0,z1, (w2,w3) -> z2,z3, (w4,w5) -> z4 (cosine branch). */
void orc_noise(uint64_t seed, uint64_t stream, double z[5])
{
    uint32_t a[4], b[4];
    draw4(seed, stream, 0u, ORC_TAG_NOISE, a);
    draw4(seed, stream, 1u, ORC_TAG_NOISE, b);
    uint32_t w[6] = {a[0], a[1], a[2], a[3], b[0], b[1]};
    for (int p = 0; p < 3; ++p) {
        double r = sqrt(-2.0 * log(orc_u01(w[2 * p])));
        double ph = 2.0 * ORC_PI * orc_u01(w[2 * p + 1]);
        z[2 * p] = r * cos(ph);
        if (2 * p + 1 < 5) z[2 * p + 1] = r * sin(ph);
    }
}

void orc_noise_batch(uint64_t seed, uint64_t id_base, int64_t n, double *z /* [5][n] */)
{
    for (int64_t i = 0; i < n; ++i) {
        double v[5];
        orc_noise(seed, id_base + (uint64_t)i, v);
        for (int d = 0; d < 5; ++d) z[d * n + i] = v[d];
    }
}

/* ------------------------------------------------------------------------------------ */
/* Analog walk through one cell (section "Monte Carlo Method", eq. 4).                     */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t face;    /* 0..3, or ORC_FACE_ABSORBED / ORC_FACE_CAPPED */
    double pos;      /* counter-clockwise position along the exit face, as a fraction of
                        that face's length, [0,1] */
    double u, v;     /* exit direction (cos, sin) in the frame of the walk */
    double len;      /* total track length in the cell, in units of the cell's height */
    uint32_t ncoll;  /* collisions (scatterings) inside the cell */
} orc_exit;

/* The cell is the rectangle [0, a] x [0, 1] (a = 1: the unit square), lengths in units of its
 * height, tau = sigma_t * height.
 * xy = 0: flatland, directions on the unit circle, isotropic scattering phi = 2 pi xi.
 * xy = 1: XY geometry (eq. 1 over the sphere, the problem invariant along z): (u, v) is the
 *          projection of a unit direction on the plane, lengths are three-dimensional; a
 *          collision draws mu = cos(polar angle) = 2 xi' - 1 and phi = 2 pi xi, giving
 *          (u, v) = sqrt(1 - mu^2) (cos phi, sin phi).
 * mode 0 ("C", continuous absorption): flights ~ Exp(sig_s) with sig_s = c * tau; the weight
 *          is attenuated analytically afterwards (eqs. 5-6), so every walk ends on a face.
 * mode 1 ("A", analog absorption): flights ~ Exp(tau); each collision absorbs with
 *          probability 1 - c (xi > c), otherwise scatters. */
void orc_walk(double tau, double c, int mode, int xy, double a, double x, double y, double u,
              double v, uint64_t seed, uint64_t stream, orc_exit *e)
{
    const double sig = (mode == 0) ? c * tau : tau;
    double len = 0.0;
    uint32_t n = 0;
    for (uint32_t flight = 0;; ++flight) {
        if (flight >= ORC_MAX_FLIGHTS) {
            e->face = ORC_FACE_CAPPED; e->pos = 0.0; e->u = u; e->v = v; e->len = len; e->ncoll = n;
            return;
        }
        /* distance to the cell boundary along (u, v) */
        double tx = INFINITY, ty = INFINITY;
        if (u > 0.0) tx = (a - x) / u; else if (u < 0.0) tx = -x / u;
        if (v > 0.0) ty = (1.0 - y) / v; else if (v < 0.0) ty = -y / v;
        int xface = (tx <= ty);
        double db = xface ? tx : ty;
        if (db < 0.0) db = 0.0;

        uint32_t r[4];
        draw4(seed, stream, flight, ORC_TAG_WALK, r);
        double ds = (sig > 0.0) ? -log(orc_u01(r[0])) / sig : INFINITY;   /* eq. 4 */

        if (ds >= db) {               /* streams to the boundary and leaves the cell */
            len += db;
            int face;
            double pos;
            if (xface) {
                double ye = y + db * v;
                ye = ye < 0.0 ? 0.0 : (ye > 1.0 ? 1.0 : ye);
                if (u > 0.0) { face = 1; pos = ye; } else { face = 3; pos = 1.0 - ye; }
            } else {
                double xe = x + db * u;
                xe = xe < 0.0 ? 0.0 : (xe > a ? a : xe);
                /* bottom and top faces have length a: position as a fraction of it */
                if (v > 0.0) { face = 2; pos = (a - xe) / a; } else { face = 0; pos = xe / a; }
            }
            e->face = face; e->pos = pos; e->u = u; e->v = v; e->len = len; e->ncoll = n;
            return;
        }
        /* collision inside the cell */
        x += ds * u;
        y += ds * v;
        len += ds;
        n += 1;
        if (mode == 1 && orc_u01(r[2]) > c) {
            e->face = ORC_FACE_ABSORBED; e->pos = 0.0; e->u = u; e->v = v; e->len = len; e->ncoll = n;
            return;
        }
        double phi = 2.0 * ORC_PI * orc_u01(r[1]);   /* isotropic scattering */
        u = cos(phi);
        v = sin(phi);
        if (xy) {                                      /* on the sphere, projected */
            double mu = 2.0 * orc_u01(r[3]) - 1.0;
            double st = sqrt(1.0 - mu * mu);
            u *= st;
            v *= st;
        }
    }
}

/* Batch of canonical transmissions: particle i enters the left face at (0, y_in[i]) with
 * direction (sqrt(1 - s^2), s), s = sin_th[i], in a cell of optical side exp(log_tau[i]) and
 * scattering ratio c[i]; random stream id_base + i.  Outputs are [n] arrays. */
typedef struct {
    const float *log_tau, *c, *y_in, *sin_th;
    const float *x_in, *cos_phi;   /* births inside the cell (internal model), else NULL */
    const float *log_aspect;        /* rectangular cells [0, A] x [0, 1], else NULL */
    const float *omega_x;           /* XY geometry: in-plane x component of the entry
                                       direction (sin_th holds the y component), else NULL */
    int64_t n;
    int mode;
    uint64_t seed, id_base;
    int32_t *face;
    double *pos, *u, *v, *len;
    uint32_t *ncoll;
    int64_t begin, end;
} walk_job;

static void *walk_worker(void *arg)
{
    walk_job *j = (walk_job *)arg;
    for (int64_t i = j->begin; i < j->end; ++i) {
        double s = (double)j->sin_th[i];
        double x0 = 0.0, u0 = j->omega_x ? (double)j->omega_x[i] : sqrt(1.0 - s * s);
        if (j->x_in) {            /* birth at (x, y) with direction (cos phi, sin phi) */
            x0 = (double)j->x_in[i];
            u0 = (double)j->cos_phi[i];
        }
        double a = j->log_aspect ? exp((double)j->log_aspect[i]) : 1.0;
        orc_exit e;
        orc_walk(exp((double)j->log_tau[i]), (double)j->c[i], j->mode, j->omega_x != NULL, a, x0,
                 (double)j->y_in[i], u0, s, j->seed, j->id_base + (uint64_t)i, &e);
        j->face[i] = e.face; j->pos[i] = e.pos; j->u[i] = e.u; j->v[i] = e.v;
        j->len[i] = e.len; j->ncoll[i] = e.ncoll;
    }
    return NULL;
}

static void run_walks(const float *log_tau, const float *c, const float *y_in, const float *sin_th,
                      const float *x_in, const float *cos_phi, const float *log_aspect,
                      const float *omega_x, int64_t n, int mode, uint64_t seed,
                      uint64_t id_base, int32_t *face, double *pos, double *u, double *v, double *len,
                      uint32_t *ncoll, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    walk_job jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) {
        walk_job j = {log_tau, c, y_in, sin_th, x_in, cos_phi, log_aspect, omega_x, n, mode, seed,
                      id_base, face, pos, u, v, len, ncoll, n * t / nthreads, n * (t + 1) / nthreads};
        jobs[t] = j;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, walk_worker, &jobs[t]);
    walk_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* log_aspect may be NULL (square cells); omega_x may be NULL (flatland) or give the in-plane x
 * component of each entry direction (XY geometry; sin_th is then its y component). */
void orc_mc_transmit(const float *log_tau, const float *c, const float *y_in, const float *sin_th,
                     const float *log_aspect, const float *omega_x, int64_t n, int mode, uint64_t seed,
                     uint64_t id_base, int32_t *face, double *pos, double *u, double *v, double *len,
                     uint32_t *ncoll, int nthreads)
{
    run_walks(log_tau, c, y_in, sin_th, NULL, NULL, log_aspect, omega_x, n, mode, seed, id_base, face,
              pos, u, v, len, ncoll, nthreads);
}

/* First-flight split of a batch of canonical transmissions: particle i crosses its cell without
 * a collision with probability exp(-c tau d_b), d_b the length of its entry ray to the boundary
 * (flights ~ Exp(c tau), eq. 4); the decision compares it with xi = u01(word 0) of
 * Philox(seed, (id lo, id hi, 0, 4)), id = id_base + i.  flag[i] = 1 for an uncollided crossing,
 * whose exit is the ray's end (the straight walk through a cell without scattering). */
void orc_uncollided_split(const float *log_tau, const float *c, const float *y_in, const float *sin_th,
                          const float *log_aspect, const float *omega_x, int64_t n, uint64_t seed,
                          uint64_t id_base, int32_t *flag, int32_t *face, double *pos, double *u,
                          double *v, double *len)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = (double)sin_th[i];
        double u0 = omega_x ? (double)omega_x[i] : sqrt(1.0 - s * s);
        double a = log_aspect ? exp((double)log_aspect[i]) : 1.0;
        double tau = exp((double)log_tau[i]);
        orc_exit e;
        /* no scattering: one flight to the boundary */
        orc_walk(0.0, 0.0, 0, omega_x != NULL, a, 0.0, (double)y_in[i], u0, s, seed, id_base + (uint64_t)i, &e);
        double pu = exp(-(double)c[i] * tau * e.len);
        uint32_t r[4];
        draw4(seed, id_base + (uint64_t)i, 0u, ORC_TAG_SPLIT, r);
        flag[i] = orc_u01(r[0]) <= pu;
        face[i] = e.face; pos[i] = e.pos; u[i] = e.u; v[i] = e.v; len[i] = e.len;
    }
}

/* Batch of walks started inside the cell: particle i is born at (x[i], y[i]) with direction
 * (cos_phi[i], sin_phi[i]) (the walk that the internal, volumetric-source model replaces). */
void orc_mc_transmit_internal(const float *log_tau, const float *c, const float *x, const float *y,
                              const float *cos_phi, const float *sin_phi, int64_t n, int mode,
                              uint64_t seed, uint64_t id_base, int32_t *face, double *pos, double *u,
                              double *v, double *len, uint32_t *ncoll, int nthreads)
{
    run_walks(log_tau, c, y, sin_phi, x, cos_phi, NULL, NULL, n, mode, seed, id_base, face, pos, u, v,
              len, ncoll, nthreads);
}

/* Canonical transmissions with FP64 conditions and explicit random stream ids (the transport
 * composition of the oracle): particle i enters the left face of the cell [0, a[i]] x [0, 1] at
 * height y[i] with direction (u[i], s[i]) (flatland: u = sqrt(1 - s^2); XY geometry: the
 * in-plane projection), optical height tau[i], scattering ratio c[i], stream ids[i].
 *   orc_noise_ids:  z ~ N(0, I_5) of stream ids[i] (orc_noise), [5][n]
 *   orc_walk_ids:   the mode-C analog walk (orc_walk)
 *   orc_split_ids:  the first-flight split of orc_uncollided_split (flag, and the entry ray's
 *                   exit for every particle) */
void orc_noise_ids(uint64_t seed, const uint64_t *ids, int64_t n, double *z /* [5][n] */)
{
    for (int64_t i = 0; i < n; ++i) {
        double v[5];
        orc_noise(seed, ids[i], v);
        for (int d = 0; d < 5; ++d) z[d * n + i] = v[d];
    }
}

void orc_walk_ids(const double *tau, const double *c, const double *y, const double *u, const double *s,
                  const double *a, int xy, int64_t n, uint64_t seed, const uint64_t *ids, int32_t *face,
                  double *pos, double *eu, double *ev, double *len)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_exit e;
        orc_walk(tau[i], c[i], 0, xy, a[i], 0.0, y[i], u[i], s[i], seed, ids[i], &e);
        face[i] = e.face; pos[i] = e.pos; eu[i] = e.u; ev[i] = e.v; len[i] = e.len;
    }
}

void orc_split_ids(const double *tau, const double *c, const double *y, const double *u, const double *s,
                   const double *a, int xy, int64_t n, uint64_t seed, const uint64_t *ids, int32_t *flag,
                   int32_t *face, double *pos, double *eu, double *ev, double *len, double *margin)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_exit e;
        orc_walk(0.0, 0.0, 0, xy, a[i], 0.0, y[i], u[i], s[i], seed, ids[i], &e);
        double pu = exp(-c[i] * tau[i] * e.len);
        uint32_t r[4];
        draw4(seed, ids[i], 0u, ORC_TAG_SPLIT, r);
        flag[i] = orc_u01(r[0]) <= pu;
        if (margin) margin[i] = fabs(orc_u01(r[0]) - pu);
        face[i] = e.face; pos[i] = e.pos; eu[i] = e.u; ev[i] = e.v; len[i] = e.len;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Cell-to-cell transport with the track-length estimator (eqs. 5-7, section "Transport   */
/* Algorithm"), analog mode-C walk inside every cell.                                      */
/* ------------------------------------------------------------------------------------ */

/* Rotation by k quarter turns counter-clockwise. */
static void rot(int k, double a, double b, double *ra, double *rb)
{
    switch (k & 3) {
    case 0: *ra = a; *rb = b; break;
    case 1: *ra = -b; *rb = a; break;
    case 2: *ra = -a; *rb = -b; break;
    default: *ra = b; *rb = -a; break;
    }
}

typedef struct {
    int32_t nx, ny;
    double L, Ly;               /* cell width (along x) and height (along y) */
    const double *tau, *c;      /* per cell, index j * nx + i; tau = sigma_t * L (the width) */
    int32_t src_x0, src_y0, src_nx, src_ny;
    int32_t reflect;            /* 0 vacuum, 1 specular reflection at the domain boundary */
    double w_min;               /* weight cutoff */
    int32_t src_face;           /* -1 volumetric source; 0..3 isotropic incident flux on that side */
    int32_t xy;                 /* 0 flatland, 1 XY geometry (directions on the sphere) */
    uint32_t max_visits;        /* a history still alive on reaching this cell visit number ends
                                 * there, its weight tallied as cutoff */
} orc_problem;

typedef struct {
    double *flux;               /* [n_cells] sum of track-length estimates (eq. 7), per history */
    double *absorbed;           /* [n_cells] deposited weight (eq. 6) */
    double *wpath;              /* [n_cells] sum of entry weight times physical track length */
    double *path;               /* [n_cells] sum of physical track lengths */
    double *visits;             /* [n_cells] number of cell visits */
    double leak, cutoff;        /* weight leaving the domain / killed by the cutoff */
    double events;              /* number of cell transmissions sampled (incl. birth legs) */
} orc_tally;

/* Stage 3 of the transport loop for one cell visit: attenuate and tally (flux, deposit, and the
 * visit's track length: w_in * l, l and one visit). Returns w_out.
 * len_units is the track length in units of `unit` (the length of the face the walk's frame
 * took as its height). */
static double visit_tally(const orc_problem *p, int cell, double w_in, double len_units,
                          double unit, orc_tally *t)
{
    double sig_a = (1.0 - p->c[cell]) * p->tau[cell] / p->L;
    double ls = len_units * unit;                    /* physical track length */
    double dw = w_in * (-expm1(-sig_a * ls));        /* eq. 6 */
    double V = p->L * p->Ly;
    double phi = (sig_a > 0.0) ? dw / (V * sig_a)    /* eq. 7 */
                               : w_in * ls / V;      /* sigma_a -> 0 limit of eq. 7 */
    t->flux[cell] += phi;
    t->absorbed[cell] += dw;
    t->wpath[cell] += w_in * ls;
    t->path[cell] += ls;
    t->visits[cell] += 1.0;
    return w_in - dw;
}

/* Inward direction through side f of a cell for an entry angle theta measured from the
 * inward normal, counter-clockwise positive (the canonical frame of entry side f, turned
 * back to the global frame): written out per side rather than through rot(). */
static void inward_direction(int f, double cth, double sth, double *gx, double *gy)
{
    switch (f) {
    case 3: *gx = cth; *gy = sth; break;      /* left side: normal +x */
    case 0: *gx = -sth; *gy = cth; break;     /* bottom side: normal +y */
    case 1: *gx = -cth; *gy = -sth; break;    /* right side: normal -x */
    default: *gx = sth; *gy = -cth; break;    /* top side: normal -y */
    }
}

/* The state of a history between cell visits. */
typedef struct {
    int ci, cj;                 /* current cell */
    int face;                   /* after a visit: the global exit face */
    int entry;                  /* at an entry: the global entry face */
    double pos;                 /* after a visit: counter-clockwise exit position */
    double y_in;                /* at an entry: canonical entry height */
    double gx, gy;              /* global direction */
    double w;                   /* weight */
    uint32_t event;             /* cell visit index */
} orc_state;

/* Birth of history h.  Volumetric source: a uniformly picked cell of the source block, a
 * uniform point and an isotropic direction, and the first leg in that cell by the analog walk
 * (cell visit 0), tallied; the state is the leg's exit.  Surface source: the entry into a
 * uniformly picked strip cell (cell visit 1), nothing tallied.  Returns 1 when the history is at
 * the entry of its cell (surface source), 0 when it has just finished a visit. */
static int birth(const orc_problem *p, uint64_t seed, uint32_t h, orc_tally *t, orc_state *st)
{
    /* birth: uniform cell of the source block (or strip) */
    uint32_t r[4];
    draw4(seed, (uint64_t)h, 0u, ORC_TAG_SOURCE, r);
    uint32_t nsrc = (uint32_t)(p->src_nx * p->src_ny);
    uint32_t pick = (uint32_t)(((uint64_t)r[0] * nsrc) >> 32);
    st->ci = p->src_x0 + (int)(pick % (uint32_t)p->src_nx);
    st->cj = p->src_y0 + (int)(pick / (uint32_t)p->src_nx);
    int cell = st->cj * p->nx + st->ci;
    st->w = 1.0;
    st->pos = 0.0;
    st->y_in = 0.0;
    st->event = 0;
    st->face = 0;
    st->entry = 0;

    if (p->src_face >= 0) {
        /* surface source: enter through side src_face at a uniform canonical height with the
         * cosine law for the angle to the inward normal (sin theta uniform on (-1, 1)); the
         * first transmission is this cell's, cell visit 1 */
        st->entry = p->src_face;
        st->y_in = u01_open(r[1]);
        if (p->xy) {
            /* isotropic incident flux in three dimensions: the cosine of the angle to the
             * inward normal is sqrt(xi) (pdf 2 cos over the hemisphere), the azimuth about the
             * normal psi = 2 pi xi'; the in-plane components are (sqrt(xi), sqrt(1 - xi) cos psi) */
            double xi = u01_open(r[2]);
            double psi = 2.0 * ORC_PI * orc_u01(r[3]);
            inward_direction(st->entry, sqrt(xi), sqrt(1.0 - xi) * cos(psi), &st->gx, &st->gy);
        } else {
            double s = 2.0 * u01_open(r[2]) - 1.0;
            inward_direction(st->entry, sqrt(1.0 - s * s), s, &st->gx, &st->gy);
        }
        st->event = 1;
        return 1;
    }
    /* volumetric source: uniform point, isotropic direction; first leg by the analog walk
     * from the interior birth point in the cell's own frame [0, L / Ly] x [0, 1] (lengths
     * in units of the height Ly), cell visit 0 */
    double ry = p->Ly / p->L;                        /* 1 for square cells */
    double a = p->L / p->Ly;
    double x = a * u01_open(r[1]), y = u01_open(r[2]);
    double phi = 2.0 * ORC_PI * orc_u01(r[3]);
    double sth = 1.0;
    if (p->xy) {             /* isotropic on the sphere: mu from a second draw */
        uint32_t r2[4];
        draw4(seed, (uint64_t)h, 1u, ORC_TAG_SOURCE, r2);
        double mu = 2.0 * orc_u01(r2[0]) - 1.0;
        sth = sqrt(1.0 - mu * mu);
    }
    orc_exit e;
    orc_walk(p->tau[cell] * ry, p->c[cell], 0, p->xy, a, x, y, sth * cos(phi), sth * sin(phi), seed,
             (uint64_t)h | ((uint64_t)st->event << 32), &e);
    t->events += 1.0;
    st->face = e.face;
    st->pos = e.pos;
    st->gx = e.u; st->gy = e.v;
    st->w = visit_tally(p, cell, st->w, e.len, p->Ly, t);
    return 0;
}

static void one_history(const orc_problem *p, uint64_t seed, uint32_t h, orc_tally *t)
{
    orc_state st;
    const int at_entry = birth(p, seed, h, t, &st);
    int ci = st.ci, cj = st.cj;
    int cell = cj * p->nx + ci;
    double gx = st.gx, gy = st.gy, w = st.w, pos = st.pos, y_in = st.y_in;
    uint32_t event = st.event;
    int face = st.face, entry = st.entry;
    orc_exit e;

    int entering = at_entry;                /* already at the entry of its first cell */
    for (;;) {
        if (!entering) {
            if (w < p->w_min) { t->cutoff += w; return; }
            /* stage 4: move to the neighbour through `face` */
            int ni = ci, nj = cj;
            if (face == 0) nj -= 1; else if (face == 1) ni += 1; else if (face == 2) nj += 1; else ni -= 1;
            if (ni < 0 || nj < 0 || ni >= p->nx || nj >= p->ny) {
                if (!p->reflect) { t->leak += w; return; }
                /* specular reflection: re-enter the same cell through the same face */
                ni = ci; nj = cj;
                entry = face;
                y_in = 1.0 - pos;
                if (face == 0 || face == 2) gy = -gy; else gx = -gx;
            } else {
                entry = (face + 2) & 3;
                y_in = pos;
            }
            ci = ni; cj = nj;
            cell = cj * p->nx + ci;
            event += 1;
            if (event >= p->max_visits) { t->cutoff += w; return; }
        }
        entering = 0;
        /* stage 1: rotate into the canonical left-entry frame */
        int k = (entry + 1) & 3;
        double U, Vc;
        rot(-k & 3, gx, gy, &U, &Vc);
        double s = Vc, U0 = U;
        if (!p->xy) {            /* flatland: unit direction, the x component from the y one */
            if (s > 1.0) s = 1.0;
            if (s < -1.0) s = -1.0;
            U0 = sqrt(1.0 - s * s);
        }
        /* the canonical cell: the entry face as height, the other side as width; left and
         * right faces have length Ly, bottom and top length L */
        double h_e = (entry & 1) ? p->Ly : p->L, w_e = (entry & 1) ? p->L : p->Ly;
        double rh = (entry & 1) ? p->Ly / p->L : 1.0;     /* tau scale: h_e / L */
        /* stage 2: sample the cell transmission (analog stand-in for the network) */
        orc_walk(p->tau[cell] * rh, p->c[cell], 0, p->xy, w_e / h_e, 0.0, y_in, U0, s, seed,
                 (uint64_t)h | ((uint64_t)event << 32), &e);
        t->events += 1.0;
        /* stage 3: absorption and tally */
        w = visit_tally(p, cell, w, e.len, h_e, t);
        /* back to the global frame */
        face = (e.face + k) & 3;
        pos = e.pos;
        rot(k, e.u, e.v, &gx, &gy);
    }
}

typedef struct {
    const orc_problem *p;
    uint64_t seed;
    uint32_t h0, h1;
    orc_tally t;
} tr_job;

static void *tr_worker(void *arg)
{
    tr_job *j = (tr_job *)arg;
    for (uint32_t h = j->h0; h < j->h1; ++h) one_history(j->p, j->seed, h, &j->t);
    return NULL;
}

/* Runs histories [h_begin, h_end).  Tallies are sums over histories (the caller divides by the
 * number of source particles).  out_scalars = {leak, cutoff, events}; path_out (NULL or
 * [3][n_cells]) = the path tallies: sum of w_in * l, sum of l, visits. */
void orc_transport(int32_t nx, int32_t ny, double L, double Ly, const double *tau, const double *c,
                   int32_t src_x0, int32_t src_y0, int32_t src_nx, int32_t src_ny, int32_t reflect,
                   int32_t src_face, int32_t xy, double w_min, uint64_t seed, uint32_t h_begin,
                   uint32_t h_end, double *flux, double *absorbed, double *out_scalars, int nthreads,
                   uint32_t max_visits, double *path_out)
{
    if (!(Ly > 0.0)) Ly = L;                          /* square cells */
    if (max_visits == 0) max_visits = 1u << 24;
    orc_problem p = {nx, ny, L, Ly, tau, c, src_x0, src_y0, src_nx, src_ny, reflect, w_min, src_face,
                     xy ? 1 : 0, max_visits};
    int ncell = nx * ny;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    tr_job jobs[256];
    pthread_t th[256];
    uint64_t nh = (uint64_t)(h_end - h_begin);
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].p = &p;
        jobs[t].seed = seed;
        jobs[t].h0 = h_begin + (uint32_t)(nh * (uint64_t)t / (uint64_t)nthreads);
        jobs[t].h1 = h_begin + (uint32_t)(nh * (uint64_t)(t + 1) / (uint64_t)nthreads);
        jobs[t].t.flux = (double *)calloc((size_t)ncell, sizeof(double));
        jobs[t].t.absorbed = (double *)calloc((size_t)ncell, sizeof(double));
        jobs[t].t.wpath = (double *)calloc((size_t)ncell, sizeof(double));
        jobs[t].t.path = (double *)calloc((size_t)ncell, sizeof(double));
        jobs[t].t.visits = (double *)calloc((size_t)ncell, sizeof(double));
        jobs[t].t.leak = jobs[t].t.cutoff = jobs[t].t.events = 0.0;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, tr_worker, &jobs[t]);
    tr_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    memset(flux, 0, sizeof(double) * (size_t)ncell);
    memset(absorbed, 0, sizeof(double) * (size_t)ncell);
    if (path_out) memset(path_out, 0, 3 * sizeof(double) * (size_t)ncell);
    out_scalars[0] = out_scalars[1] = out_scalars[2] = 0.0;
    for (int t = 0; t < nthreads; ++t) {
        for (int i = 0; i < ncell; ++i) {
            flux[i] += jobs[t].t.flux[i];
            absorbed[i] += jobs[t].t.absorbed[i];
            if (path_out) {
                path_out[i] += jobs[t].t.wpath[i];
                path_out[ncell + i] += jobs[t].t.path[i];
                path_out[2 * ncell + i] += jobs[t].t.visits[i];
            }
        }
        out_scalars[0] += jobs[t].t.leak;
        out_scalars[1] += jobs[t].t.cutoff;
        out_scalars[2] += jobs[t].t.events;
        free(jobs[t].t.flux);
        free(jobs[t].t.absorbed);
        free(jobs[t].t.wpath);
        free(jobs[t].t.path);
        free(jobs[t].t.visits);
    }
}

/* Births of histories [h_begin, h_end) (the source stage of orc_transport) for the oracle's
 * transport composition: state[9][n] per history = {at entry (1: surface source, the entry of
 * its cell; 0: volumetric, the exit of its first leg), cell index, face (exit face, or the
 * entry face at an entry), pos (exit position, or the canonical entry height), gx, gy, w,
 * event, 0}; the birth legs' tallies are added to flux, absorbed, path_out ([3][n_cells]) and
 * scalars[2] (events). */
void orc_birth_states(int32_t nx, int32_t ny, double L, double Ly, const double *tau, const double *c,
                      int32_t src_x0, int32_t src_y0, int32_t src_nx, int32_t src_ny, int32_t reflect,
                      int32_t src_face, int32_t xy, double w_min, uint64_t seed, uint32_t h_begin,
                      uint32_t h_end, double *state, double *flux, double *absorbed, double *path_out,
                      double *scalars)
{
    if (!(Ly > 0.0)) Ly = L;
    orc_problem p = {nx, ny, L, Ly, tau, c, src_x0, src_y0, src_nx, src_ny, reflect, w_min, src_face,
                     xy ? 1 : 0, 1u << 24};
    int ncell = nx * ny;
    orc_tally t = {flux, absorbed, path_out, path_out + ncell, path_out + 2 * ncell, 0.0, 0.0, 0.0};
    int64_t n = (int64_t)(h_end - h_begin);
    for (int64_t i = 0; i < n; ++i) {
        orc_state st;
        int at_entry = birth(&p, seed, h_begin + (uint32_t)i, &t, &st);
        double v[9] = {(double)at_entry, (double)(st.cj * nx + st.ci), (double)(at_entry ? st.entry : st.face),
                       at_entry ? st.y_in : st.pos, st.gx, st.gy, st.w, (double)st.event, 0.0};
        for (int k = 0; k < 9; ++k) state[k * n + i] = v[k];
    }
    scalars[2] += t.events;
}
