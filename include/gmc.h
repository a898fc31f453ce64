/*
 * gmc.h -- C ABI of the MI355X (gfx950) Generative Monte Carlo cell-transmission library.
 *
 * Method: Farmer, Murray, Krotz, McClarren, "Generative Monte Carlo Sampling for
 * Constant-Cost Particle Transport", arXiv 2512.13965.  A particle entering a cell is
 * "teleported" to its exit state by integrating a conditional flow-matching velocity field
 * from Gaussian noise (section "Conditional Flow Matching", eq. 8) instead of following its
 * random walk (section "Monte Carlo Method", eq. 4).  Both samplers live behind this ABI.
 *
 * Conventions for every entry point
 *   - Pointers named "device" are HIP device pointers owned by the caller; the library never
 *     frees them.  Host pointers are read before the call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every sampling call is
 *     asynchronous on that stream and returns once its kernels are enqueued.
 *   - Return value: GMC_OK (0) or a negative gmc_status; no exceptions cross the ABI and the
 *     library never aborts.  gmc_last_error() gives a thread-local message for the last
 *     failure on the calling thread.
 *   - Lengths are in units of the entry face (the cell side L for square cells) and
 *     directions are in the canonical frame in which the particle enters through the left
 *     face x = 0 of the cell [0, A] x [0, 1] (A = 1: the unit square; section "Transport
 *     Algorithm", first stage).  Faces: 0 bottom (y=0), 1 right (x=A), 2 top (y=1), 3 left
 *     (x=0).  The position along an exit face runs counter-clockwise, as a fraction of that
 *     face's length: bottom x/A, right y, top (A-x)/A, left 1-y.  Directions are unit in-plane
 *     vectors (flatland, the default) or projections of unit vectors on the sphere (XY
 *     geometry, see gmc_cond.omega_x).
 *   - Results are a pure function of (weights, condition, seed, particle id, K): they do not
 *     depend on the batch size or on a particle's position in the batch.
 */
#ifndef GMC_H
#define GMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GMC_OK = 0,
    GMC_EINVAL = -1,         /* bad argument (null pointer, size, unsupported K, bad blob) */
    GMC_ENOMEM = -2,         /* device allocation failed or a capacity would be exceeded */
    GMC_EDEVICE = -3,        /* a HIP call or kernel launch failed */
    GMC_EUNSUPPORTED = -4    /* valid request the library does not implement (e.g. width) */
} gmc_status;

typedef enum {
    GMC_FP32 = 0,            /* FP32 operands, FP32 MFMA */
    GMC_BF16 = 1,            /* BF16 operands, FP32 accumulation */
    GMC_FP8_E4M3 = 2         /* OCP e4m3 hidden layers (per-layer power-of-two scales),
                                first and last layer BF16, FP32 accumulation */
} gmc_precision;

typedef enum { GMC_MODE_CONTINUOUS = 0, GMC_MODE_ANALOG = 1 } gmc_walk_mode;
typedef enum { GMC_SAMPLER_GMC = 0, GMC_SAMPLER_MC = 1 } gmc_sampler;
/* ODE integrator of the generative sampler: explicit Euler (one network evaluation per step,
 * eq. 8 as written) or the classic fourth-order Runge-Kutta scheme (four evaluations per step;
 * the integrator behind the timings of the paper section "Convergence and Performance", 12 steps). */
typedef enum { GMC_EULER = 0, GMC_RK4 = 1 } gmc_integrator;

#define GMC_FACE_ABSORBED (-1)   /* analog-absorption walk ended inside the cell */
#define GMC_FACE_CAPPED (-2)     /* walk exceeded 2^24 flights (never seen in practice) */

/* Canonical entry conditions of n transmissions, device SoA, float32 [n] each
 * (paper eq. 10 in the reading ln tau = ln(sigma_t L), c = sigma_s / sigma_t, with the
 * rectangle's optical width and height W~, H~ given as H~ = tau and W~ / H~ = A):
 *   log_tau     natural log of the optical length tau = sigma_t * L of the entry face
 *   c           scattering ratio sigma_s / sigma_t in [0, 1]
 *   y_in        entry height on the left face, as a fraction of its length, in [0, 1]
 *   sin_th      sine of the entry angle from +x, in (-1, 1) (the direction is
 *               (sqrt(1 - sin_th^2), sin_th))
 *   log_aspect  optional (NULL: square cells): ln A, A = cell width along +x over the entry
 *               face's length; the canonical cell is [0, A] x [0, 1] in units of the entry
 *               face, exit positions are fractions of the exit face's length and path lengths
 *               are in units of the entry face
 *   omega_x     optional (NULL: flatland): XY geometry (eq. 1 over the sphere, the problem
 *               invariant along z); the entry direction's in-plane projection is
 *               (omega_x, sin_th), inside the unit disk, and paths are three-dimensional */
typedef struct {
    const float *log_tau, *c, *y_in, *sin_th;
    const float *log_aspect;
    const float *omega_x;
} gmc_cond;

/* Birth conditions of n particles born inside a cell (the internal, volumetric-source model of
 * the paper section "Network Architecture and Inputs": the condition holds the two-dimensional
 * birth position and the birth direction), device SoA, float32 [n] each, in the cell's own
 * frame (no canonical rotation: the exit face is reported in the cell's orientation):
 *   log_tau, c         as in gmc_cond
 *   x, y               birth position in the unit cell, (0, 1) each
 *   cos_phi, sin_phi   birth direction (unit vector) */
typedef struct {
    const float *log_tau, *c, *x, *y, *cos_phi, *sin_phi;
} gmc_cond_internal;

/* Exit records of n transmissions, device SoA, [n] each (paper eq. 11):
 *   face     int32 exit face 0..3 (GMC_FACE_* for walks that did not exit; -1 also for a
 *            generative sample whose network state left the decodable range, see gmc_transmit)
 *   pos      float32 counter-clockwise position along the exit face, [0, 1]
 *   dir_cos, dir_sin   float32 exit direction (unit vector, pointing out of the face)
 *   path     float32 total track length in the cell, units of L */
typedef struct {
    int32_t *face;
    float *pos, *dir_cos, *dir_sin, *path;
} gmc_exit;

typedef struct gmc_model gmc_model;

/* Per-device set-up of the current device: queries its compute units and allocates the ring of
 * 4096 work counters (32 KiB) that mc_transmit and mc_transmit_internal launches take in turn
 * (kept until the process ends).  Needed once per device before those calls, which allocate
 * nothing themselves (GMC_EINVAL if the device was not set up); gmc_model_create and
 * gmc_world_create do it for their device.  Idempotent and thread-safe.  Errors: GMC_EDEVICE,
 * GMC_ENOMEM, GMC_EUNSUPPORTED (device index beyond 63). */
int gmc_device_init(void);

/* Parses a weights blob and uploads it to the current device in the layout the kernels read.
 * Blob (little-endian): "GMCW0001", u32 version=1, n_in=10, hidden H, n_out=5, n_layers=5,
 * flags, seed, reserved; f32 act_scale[5], w_scale[5]; then per layer l = 1..5 the float32
 * weight matrix W_l[out][in] (row-major) followed by the float32 bias b_l[out].  Layer dims:
 * 10->H, H->H (x3), H->5.  Network input order: [x0..x4, t, ln tau, c, 2*y_in-1, sin_th];
 * SiLU after layers 1..4 (paper section "Network Architecture and Inputs", eqs. 10-11).
 * Supported: H in {128, 256} for GMC_FP32, H in {128, 256, 512} for GMC_BF16 / GMC_FP8_E4M3.
 * flags: bit 0 XY geometry (n_in = 11, condition ln tau, c, 2 y_in - 1, omega_y, omega_x);
 * bit 1 a boundary model fitted on collided crossings only (the transport step then places
 * uncollided crossings itself, see gmc_uncollided_split); bit 2 the residual network with
 * adaptive modulation (below); other bits GMC_EINVAL.
 * GMC_BF16 and GMC_FP8_E4M3 models of the plain network are evaluated with their hidden
 * activations scaled by -log2(e): the first layer's weights and the hidden biases are multiplied
 * by -log2(e) and the output layer's weights by -ln 2 (float32 products) before the BF16
 * rounding (the same network in exact arithmetic).  The e4m3 layers keep their weights and take
 * half the scaled activation over their activation scale (so e4m3's limit of 448 leaves the
 * plain SiLU's headroom); 2 w_scale act_scale must lie in [2^-127, 2^127] (GMC_EINVAL).
 * Residual network (flag bit 2; paper "Network Architecture and Inputs": learned embeddings of
 * t and c, residual blocks with adaptive modulation): n_layers = 3 (blocks), reserved = 32
 * (embedding width E), scales 1; layers in blob order: input W_in[H][13 + n_c] over
 * [x0..x4, sin pi t, cos pi t, sin 2 pi t, ..., cos 8 pi t, condition (n_c = n_in - 6)];
 * embedding W_e[32][8 + n_c] over [time features, condition] with SiLU; per block the main map
 * A[H][H], the scale map G[H][32] and the shift map S[H][32] (h += SiLU((1 + G e + g) *
 * (A h + a) + S e + s)); output W_o[5][H].  Supported: H = 128 for GMC_FP32, H in
 * {128, 256, 512} for GMC_BF16 (BF16: the residual stream is stored in BF16); FP8
 * GMC_EUNSUPPORTED.
 * The scales must be positive powers of two.  The blob is host memory owned by the caller.
 * On success *out owns device memory until gmc_model_destroy(). */
int gmc_model_create(const void *host_blob, size_t nbytes, int precision, gmc_model **out);
int gmc_model_destroy(gmc_model *m);
/* Reports the hidden width and precision of a model (either pointer may be NULL). */
int gmc_model_info(const gmc_model *m, int *hidden, int *precision);
/* Reports the network's input width: 10 for a boundary model of square cells (gmc_cond
 * without log_aspect), 11 for a boundary model of rectangular cells (input order [x0..x4, t,
 * ln tau, c, 2 y_in - 1, sin th, ln A]), 12 for an internal model (gmc_cond_internal; input
 * order [x0..x4, t, ln tau, c, 2x - 1, 2y - 1, cos phi, sin phi]). */
int gmc_model_inputs(const gmc_model *m, int *n_in);

/* Samples n cell transmissions with the generative sampler (paper "Transport Algorithm",
 * second stage; eq. 8): x(0) = z ~ N(0, I_5); K explicit Euler steps x += v(x, k/K | c) / K;
 * the exit record is decoded from x_K (eq. 11: a0 = 2*pos - 1, (a1, a2) = direction,
 * a3 = ln path, face = number of thresholds -1, 0, 1 reached by a4; position clamped to
 * [0, 1]; direction normalised and its normal component reflected if it points into the
 * cell; outward normal if its norm is below 1e-6).  A state x_K with a component beyond 32 in
 * magnitude, or not finite, lies outside the range the targets span (|a| <= 16) and is
 * rejected: face -1, the other fields 0 (a diverging trajectory, a few in 10^7 samples of the
 * fitted H = 128 models; the transport step drops such a particle's weight into the cutoff
 * tally).
 *   K          1..1024
 *   seed, id_base   particle i draws its noise from Philox4x32-10 with key = seed and
 *              counter (id lo, id hi, j, 1), j = 0, 1, id = id_base + i; Box-Muller pairs
 *              (w0,w1) (w2,w3) (w4,w5) give z0..z4
 *   noise_opt  NULL, or device float32 [5][n] (row d holds z_d of every particle): used
 *              instead of the generator
 *   raw_opt    NULL, or device float32 [5][n] receiving x_K before decoding
 *   out        device exit record (all five arrays required)
 * n = 0 is a no-op.  Errors: GMC_EINVAL (null pointers, K out of range), GMC_EDEVICE. */
/* m must be a boundary model: n_in = 10 takes no log_aspect (GMC_EINVAL if one is given);
 * n_in = 11 reads it (NULL: ln A = 0). */
int gmc_transmit(const gmc_model *m, gmc_cond cond, int64_t n, int K, uint64_t seed,
                 uint64_t id_base, const float *noise_opt, float *raw_opt, gmc_exit out,
                 void *stream);

/* gmc_transmit with a choice of ODE integrator over the same K uniform steps of [0, 1]:
 *   integrator GMC_EULER: identical to gmc_transmit.
 *   integrator GMC_RK4:   x_{k+1} = x_k + (h/6)(k1 + 2 k2 + 2 k3 + k4), h = 1/K, with
 *              k1 = v(x_k, t_k), k2 = v(x_k + h k1/2, t_k + h/2), k3 = v(x_k + h k2/2, t_k + h/2),
 *              k4 = v(x_k + h k3, t_k + h); t_k = k/K (4K network evaluations).
 * Other arguments, ownership and errors as for gmc_transmit; GMC_EINVAL for an unknown
 * integrator. */
int gmc_sample(const gmc_model *m, gmc_cond cond, int64_t n, int integrator, int K, uint64_t seed,
               uint64_t id_base, const float *noise_opt, float *raw_opt, gmc_exit out,
               void *stream);

/* The generative sampler for particles born inside cells (internal model, n_in = 12): the
 * same ODE, integrators, noise streams, decoding and errors as gmc_sample, with the birth
 * condition in place of the entry condition.  GMC_EINVAL if m is not an internal model. */
int gmc_sample_internal(const gmc_model *m, gmc_cond_internal cond, int64_t n, int integrator, int K,
                        uint64_t seed, uint64_t id_base, const float *noise_opt, float *raw_opt,
                        gmc_exit out, void *stream);

/* First-flight split of n canonical transmissions (an analytic variant beside the paper's single
 * model; used by the transport step with a collided-only model, blob flag bit 1): the entry ray
 * meets the cell boundary after d_b, and with flights ~ Exp(c tau) (eq. 4) the particle crosses
 * without a collision with probability exp(-c tau d_b).  Particle i compares it with
 * xi = ((w >> 8) + 1) 2^-24, w = word 0 of Philox4x32-10 with key = seed and counter
 * (id lo, id hi, 0, 4), id = id_base + i.  uncollided[i] (device int32 [n]) = 1 for an
 * uncollided crossing, whose exit record is written (face and position at the ray's end, the
 * entry direction, path d_b); 0 otherwise, the record then left as it was.  Flatland, XY
 * geometry and rectangular cells as for mc_transmit.  Errors: GMC_EINVAL, GMC_EDEVICE. */
int gmc_uncollided_split(gmc_cond cond, int64_t n, uint64_t seed, uint64_t id_base, int32_t *uncollided,
                         gmc_exit out, void *stream);

/* Samples n cell transmissions with the analog random walk that the generative sampler
 * replaces (paper "Monte Carlo Method", eq. 4) through the canonical cell [0, A] x [0, 1]
 * (A = 1 without log_aspect; lengths in units of the entry face).  With omega_x (XY geometry)
 * a scattering also draws mu = 2 xi_3 - 1 from word 3 and the new in-plane direction is
 * sqrt(1 - mu^2) (cos phi, sin phi); exit directions are then projections (norm <= 1).
 * Flights d = -ln(xi) / sigma with
 * xi = ((w >> 8) + 1) * 2^-24 in (0, 1], isotropic flatland scattering phi = 2 pi xi'.
 *   mode GMC_MODE_CONTINUOUS: sigma = c * tau (implicit capture: the caller attenuates the
 *        weight by exp(-(1 - c) tau path), eqs. 5-6); every walk ends on a face.
 *   mode GMC_MODE_ANALOG: sigma = tau, a collision absorbs when xi'' > c (face = -1).
 *   Flight j of particle i uses Philox4x32-10 with key = seed and counter
 *   (id lo, id hi, j, 2), id = id_base + i: word 0 -> flight length, 1 -> new direction,
 *   2 -> absorption test.
 *   ncoll_opt  NULL, or device uint32 [n] receiving the number of collisions in the cell.
 * Errors: GMC_EINVAL, GMC_EDEVICE. */
/* The walk's lanes take particles from a work counter of the ring gmc_device_init allocates
 * (GMC_EINVAL if the current device was not set up); the call allocates nothing. */
int mc_transmit(gmc_cond cond, int64_t n, int mode, uint64_t seed, uint64_t id_base,
                gmc_exit out, uint32_t *ncoll_opt, void *stream);
/* mc_transmit for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same walk, arguments, random
 * streams and outputs, bit for bit, but its work counter is one of 64 counters of a fixed
 * 512-byte device array that the library holds on each GPU until the process ends (its address
 * looked up by gmc_device_init, which must have run on the current device: GMC_EINVAL
 * otherwise).  The call allocates nothing, calls no allocating routine and records no memset:
 * it zeroes its counter with a kernel on `stream`.  Calls take the 64 counters in turn; calls
 * that overlap on one GPU (other streams, or more than 64 in flight) may share a counter and
 * then race.  Errors as mc_transmit, plus GMC_EINVAL for n beyond 2^62 (the counter's range). */
int mc_transmit_noalloc(gmc_cond cond, int64_t n, int mode, uint64_t seed, uint64_t id_base,
                        gmc_exit out, uint32_t *ncoll_opt, void *stream);
/* The analog walk of mc_transmit started inside the cell at (x, y) with direction
 * (cos_phi, sin_phi) (the walk the internal model replaces); same modes, random streams,
 * outputs and errors.  The first flight starts at the birth point. */
int mc_transmit_internal(gmc_cond_internal cond, int64_t n, int mode, uint64_t seed, uint64_t id_base,
                         gmc_exit out, uint32_t *ncoll_opt, void *stream);

/* Decodes raw network outputs (device float32 [5][n]) into exit records with the rule of
 * gmc_transmit.  flags_opt: NULL or device int32 [n]: bit0 position clamped, bit1 direction
 * reflected, bit2 zero-norm direction, bit3 (alone) rejected state. */
int gmc_decode(const float *raw, int64_t n, gmc_exit out, int32_t *flags_opt, void *stream);

/* ---------------------------------------------------------------------------------------- */
/* Cell-to-cell transport (paper section "Transport Algorithm", stages 1-4; track-length     */
/* flux estimator of eqs. 5-7).  A world owns one device particle bank shared by up to        */
/* max_problems problems, so particles of different problems (grids, materials, seeds) are     */
/* sampled together in one launch.                                                             */
/* ---------------------------------------------------------------------------------------- */
typedef struct gmc_world gmc_world;

/* One transport problem: nx * ny cells of width L and height Ly (physical lengths; Ly = 0 means
 * square cells, Ly = L), cell (i, j) at index j * nx + i (i along x).  tau[cell] = sigma_t * L
 * (>= 0) and c[cell] = sigma_s / sigma_t (in [0, 1]) are host FP64 arrays read during
 * gmc_problem_add.  A transmission is sampled in the canonical frame of its entry face (that
 * face as the unit of length: tau * Ly / L and aspect A = L / Ly through the left and right
 * faces, tau and A = Ly / L through the bottom and top); rectangular cells need an 11-input
 * boundary model for the generative sampler and volumetric births by the analog walk.
 * xy = 1 selects XY geometry (eq. 1 over the sphere, invariant along z): directions are
 * projections of unit directions, scattering and volumetric sources are isotropic on the sphere
 * (mu from the next Philox block of the birth stream), a surface source is isotropic incident
 * flux (cosine sqrt(xi) to the normal, azimuth psi), tracks are three-dimensional.  All problems
 * of a world share one geometry (GMC_EINVAL otherwise); the generative sampler then needs a
 * model of that geometry.  Boundaries are vacuum
 * (reflect = 0) or specular (reflect = 1).  A history ends when it leaves the domain or when its
 * weight drops below w_min after a cell visit (the weight is then tallied as cutoff), and at the
 * latest before its cell visit number max_visits (0: 2^24; otherwise at least 2), its weight
 * then tallied as cutoff too: a bound for histories that would never end (a reflecting box
 * without absorption).
 * Sources (one unit-weight particle per history):
 *   src_face = -1: isotropic volumetric source, uniform over the cells
 *     [src_x0, src_x0 + src_nx) x [src_y0, src_y0 + src_ny) (a birth picks the cell with the
 *     first Philox word, the point with the next two, the angle with the fourth);
 *   src_face = f in 0..3 (bottom, right, top, left): surface source of isotropic incident flux
 *     on that side of the domain (the hohlraum drive of the paper's second benchmark): the
 *     source cells must be a strip along that side (f = 3: src_x0 = 0, src_nx = 1; f = 1:
 *     src_x0 = nx - 1, src_nx = 1; f = 0: src_y0 = 0, src_ny = 1; f = 2: src_y0 = ny - 1,
 *     src_ny = 1) and the boundaries vacuum.  A birth enters a uniformly picked source cell
 *     through face f at a uniform height (canonical y_in) with a cosine-law direction
 *     (canonical sin theta = 2 u - 1), and its first transmission is that cell's.
 * History h draws its birth from Philox key = seed, counter (h, 0, 0, 3); the k-th cell it
 * visits (k = 0 for a volumetric birth cell; a surface birth starts at k = 1) uses random
 * stream id h + 2^32 k for its transmission. */
typedef struct {
    int32_t nx, ny;
    double L;
    const double *tau, *c;
    int32_t src_x0, src_y0, src_nx, src_ny;
    int32_t reflect;
    double w_min;
    uint64_t seed;
    int32_t src_face;
    double Ly;
    int32_t xy;
    int64_t max_visits;
} gmc_problem_desc;

/* Device bytes gmc_world_create would allocate for these capacities (admission control). */
int gmc_world_footprint(int64_t bank_capacity, int32_t max_problems, int64_t max_cells, size_t *bytes);
/* Allocates a world on the current device: a bank of bank_capacity particles (two copies, for
 * compaction), sampler staging for as many transmissions, max_problems problem slots and
 * max_cells cells of materials and FP64 tallies shared by the problems.  GMC_ENOMEM if the
 * device allocation fails. */
int gmc_world_create(int64_t bank_capacity, int32_t max_problems, int64_t max_cells, gmc_world **out);
int gmc_world_destroy(gmc_world *w);
/* Adds a problem: takes a slot and nx * ny cells, uploads the materials, zeroes its tallies.
 * Synchronises `stream`.  GMC_EINVAL for a bad grid, material or source description (see
 * gmc_problem_desc); GMC_ENOMEM when no slot or not enough contiguous free cells. */
int gmc_problem_add(gmc_world *w, const gmc_problem_desc *d, int32_t *pid, void *stream);
/* Frees a problem's slot and cells; GMC_EINVAL while it still has particles in flight. */
int gmc_problem_remove(gmc_world *w, int32_t pid);
/* Births of histories [h_begin, h_begin + count) of problem pid (ids below 2^32): source
 * sampling, and for a volumetric source the first leg in the birth cell (the analog walk with
 * continuous absorption, or the internal model set by gmc_world_set_source_model), its tally,
 * and the move to the neighbour (a surface source's births enter their cell directly).  Survivors join the bank.  GMC_ENOMEM if count exceeds
 * the free bank slots.  Synchronises `stream`; *n_alive_out (optional) = particles in flight. */
int gmc_world_inject(gmc_world *w, int32_t pid, uint64_t h_begin, int64_t count, void *stream,
                     int64_t *n_alive_out);
/* One transport step for every particle in flight: canonical conditions (stage 1), one cell
 * transmission each with the generative sampler (sampler = GMC_SAMPLER_GMC, model m, K steps
 * of the world's integrator) or the analog walk with continuous absorption (GMC_SAMPLER_MC, m unused), FP64
 * attenuation and tallies (stage 3), move / leak / cutoff and compaction (stage 4).
 * With a model fitted on collided crossings (blob flag bit 1) stage 1 first draws each
 * particle's first-flight split (gmc_uncollided_split's test and exit); only the collided
 * particles, compacted, go through the sampler, whose exits are scattered back.
 * Synchronises `stream`; *n_alive_out (optional) = particles still in flight.  GMC_EINVAL for
 * an unknown sampler, or for GMC without a boundary model (n_in = 10) or with K outside 1..1024. */
int gmc_transport_step(gmc_world *w, int sampler, const gmc_model *m, int K, void *stream,
                       int64_t *n_alive_out);
/* Streaming of uncollided crossings in steps with the first-flight split (a model fitted on
 * collided crossings): a particle whose crossing is uncollided is carried on inside the step,
 * its attenuation, tallies and move done there (FP64, global atomics), through up to
 * max_crossings cells; the step's sampler then sees it at its next collided crossing.  Every
 * crossing is decided by the same random numbers (keyed by history and cell visit) whatever
 * the value, so results are the same up to the order of FP64 additions; 1 = one crossing per
 * particle per step.  Default 64.  GMC_EINVAL outside 1..1024. */
int gmc_world_set_streaming(gmc_world *w, int max_crossings);
/* Cell transmissions carried out by gmc_transport_step since the world was created: one per
 * particle and step plus the crossings streamed inside steps (current after each step). */
int gmc_world_transmissions(const gmc_world *w, int64_t *count);
/* Source births of later gmc_world_inject calls: m = NULL (the default) walks each birth's first
 * leg with the analog walk; an internal model (n_in = 12) samples it with the generative sampler
 * instead (K steps of the world's integrator; paper "Transport Algorithm", first stage, and
 * Fig. 1a's separate network for particles born inside cells).  The model must outlive its use.
 * GMC_EINVAL if m is not an internal model or K is outside 1..1024. */
int gmc_world_set_source_model(gmc_world *w, const gmc_model *m, int K);
/* Integrator (GMC_EULER, the default, or GMC_RK4) that later gmc_transport_step calls with the
 * generative sampler use; K then counts integration steps.  GMC_EINVAL otherwise. */
int gmc_world_set_integrator(gmc_world *w, int integrator);
/* enable != 0: later gmc_transport_step calls replay a HIP graph of the step (gather, sampler,
 * counter reset, apply) captured once per (sampler, model, K, integrator, bank parity) and per
 * particle-count bucket (the next power of two >= 1024, capped at the bank capacity); the captured
 * kernels read the particle count from the device, so one graph serves every count in its bucket.
 * Graphs are captured on a stream the world owns and replayed on the caller's stream; they are
 * released with the world.  Results equal those of the uncaptured step (FP64 tallies up to the
 * order of their atomic additions).  enable = 0 returns to direct launches. */
int gmc_world_set_graphs(gmc_world *w, int enable);
/* Particles of problem pid still in flight after the last step or injection. */
int gmc_problem_alive(const gmc_world *w, int32_t pid, int64_t *n_alive);
/* Copies problem pid's FP64 tallies, summed over its histories so far, to host arrays of
 * nx * ny doubles (any pointer may be NULL): track-length flux estimate per cell (eq. 7,
 * divided by the cell volume L^2), deposited weight per cell (eq. 6), weight that leaked out
 * of the domain from each boundary cell, weight dropped by the cutoff in each cell.
 * Synchronises `stream`. */
int gmc_problem_tally(gmc_world *w, int32_t pid, double *flux, double *absorbed, double *leak,
                      double *cutoff, void *stream);
/* Copies problem pid's FP64 path tallies (paper "Transport Algorithm", third stage: the physical
 * track length of every cell visit, the quantity the flux estimator of eqs. 5-7 integrates),
 * summed over its histories so far, to host arrays of nx * ny doubles (any pointer may be NULL):
 *   wpath       sum over the visits of the cell of w_in * l_phys (entry weight times the visit's
 *               physical track length)
 *   path        sum of l_phys
 *   visits      number of visits (births' first legs, transmissions and crossings streamed by the
 *               first-flight split alike; exact up to 2^53)
 *   rejected_w  weight of the particles whose generative sample the decoder rejected in the cell
 *               (a part of the cutoff tally; see gmc_transmit)
 *   rejected_n  number of such rejections
 * Synchronises `stream`.  GMC_EINVAL for an unknown problem. */
int gmc_problem_path_tally(gmc_world *w, int32_t pid, double *wpath, double *path, double *visits,
                           double *rejected_w, double *rejected_n, void *stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char *gmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GMC_H */
