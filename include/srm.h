/*
 * srm.h -- C ABI of the MI355X (gfx950) Swelling and Random Migration (SRM)
 * library.
 *
 * SRM (Tarasovs, "Efficient generation of large-scale non-equilibrium
 * distributions of particles", Sec. 2, Algorithms 1-6) grows the particles
 * of a periodic box step by step and after each growth step moves every
 * particle by a small random displacement, rejecting moves that overlap a
 * neighbour, until the target volume fraction is reached without overlap.
 *
 * Conventions shared by every entry point:
 *  - Return value: SRM_OK (0) or a negative srm_status.  On error,
 *    srm_last_error() returns a message (thread-local, valid until the next
 *    call on the same thread).  No C++ exception crosses this boundary.
 *  - Particle arrays are structure-of-arrays in particle-id order: a
 *    position array holds dim * n doubles, x[0..n) then y[0..n) [then
 *    z[0..n)]; normals hold 3 * n doubles the same way.
 *  - mem_kind says where caller buffers live: SRM_MEM_HOST (pageable or
 *    pinned host memory) or SRM_MEM_DEVICE (device memory of the context's
 *    GPU, e.g. torch.Tensor.data_ptr()).  The caller owns every buffer it
 *    passes; the library copies inputs and writes outputs, and never keeps a
 *    caller pointer after the call returns.
 *  - A context owns all of its device memory and runs every kernel on the
 *    HIP stream given at srm_init (0 = the null stream).  Calls that return
 *    host-visible results synchronise that stream before returning.  A
 *    context is not thread-safe: calls on one context must not overlap.
 *  - Random numbers: Philox4x32-10 keyed by the 64-bit seed, counter
 *    (particle id, sweep, kind<<31 | pass<<16 | trial<<8 | call, stream), so a
 *    run is a pure function of (inputs, params, s0, sweep0): results do not
 *    depend on launch shapes, and a saved state resumes bit-exactly.
 */
#ifndef SRM_H
#define SRM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srm_ctx srm_ctx;
typedef int32_t srm_status;

enum {
    SRM_OK = 0,
    SRM_EINVAL = -1,     /* bad argument; no side effects */
    SRM_ENOMEM = -2,     /* device or host allocation failed */
    SRM_EDEVICE = -3,    /* a HIP call failed */
    SRM_EOVERLAP = -4,   /* initial configuration overlaps at s0 */
    SRM_ENOTCONV = -5,   /* max_sweeps reached before s_target */
    SRM_ECAPACITY = -6   /* output buffer too small; *count holds the need */
};

/* Particle shapes.  SRM_PLATELET: zero-thickness circular disks (exact
 * disk-disk intersection).  SRM_SPHERODISK: the thin circular platelets of
 * Sec. 3.3 as spherodisks -- every point within h of a flat core disk of
 * radius A; a particle of outer radius a = s rho has h = thick_ratio a
 * (thickness t = thick_ratio D, D = 2a) and A = a - h.  Two spherodisks
 * overlap iff the minimum distance between their core disks is at most
 * h_i + h_j (touching counts), decided within 1e-12 (A_i + A_j) of that
 * bound, where it counts as overlap. */
enum { SRM_BALL = 0, SRM_PLATELET = 1, SRM_SPHERODISK = 2 };
enum { SRM_MEM_HOST = 0, SRM_MEM_DEVICE = 1 };
enum { SRM_PASS_MAIN = 0, SRM_PASS_SHAKE = 1 };

/* Problem statement of Algorithm 1: box edges, particle set, target, the
 * swelling and migration rates c_w and c_m and the attempt counts N_k, N_l
 * (Sec. 2).  Radii are R_i = s * rho_i with a common scale s that grows from
 * s0 to s_target. */
typedef struct {
    int32_t dim;         /* 2 (disks) or 3 (spheres, platelets) */
    int32_t shape;       /* SRM_BALL, SRM_PLATELET or SRM_SPHERODISK (both 3D only) */
    int64_t n;           /* particle count, 1 <= n < 2^31 */
    double box[3];       /* periodic box edges L_a > 0 (box[2] unused in 2D) */
    double s_target;     /* final radius scale (sets the target fraction) */
    double c_w;          /* swelling step per sweep, as a fraction of s_target */
    double c_m;          /* migration step length (absolute) */
    double c_n;          /* platelet normal step (unit-vector length) */
    double thick_ratio;  /* platelet thickness / diameter: volume only for SRM_PLATELET;
                            shape and volume for SRM_SPHERODISK (0 < thick_ratio < 0.5) */
    int32_t n_k;         /* passes per sweep before a shake, 0..32767 */
    int32_t n_l;         /* trial moves per particle per pass, 0..255 */
    uint64_t seed;       /* Philox key */
} srm_params;

typedef struct {
    int32_t committed;     /* 1: the swollen state was admitted; 0: shaken */
    int32_t passes_main;   /* migration passes on the swollen copy */
    int32_t passes_shake;  /* shake passes on the committed state */
    int32_t grid[3];       /* cells per axis used by this sweep */
    int64_t sweep;         /* sweep counter after the sweep */
    double s;              /* radius scale after the sweep */
    double fraction;       /* volume fraction at s */
    int64_t n_failed_last; /* particles that rejected every trial in the last pass */
} srm_sweep_info;

typedef struct {
    int64_t sweeps;        /* sweeps run by this call */
    int64_t passes;        /* migration passes (main + shake) */
    int64_t shakes;        /* sweeps that ended in a shake */
    int64_t updates;       /* particle updates = n * passes */
    double s, fraction;    /* final radius scale and volume fraction */
} srm_run_info;

/* Create a context.  p: parameters (copied).  pos: dim*n SoA positions in
 * [0, L_a) per axis.  rho: n shape radii > 0, or NULL for all 1.
 * normals: 3*n unit normals (platelets), else NULL.  s0: starting radius
 * scale; sweep0: starting sweep counter (resume, < 2^32).  stream: hipStream_t or
 * NULL.  Fails with SRM_EOVERLAP if two particles overlap at s0 (Algorithm 1
 * starts from a non-overlapping set), SRM_EINVAL on a bad parameter or a
 * coordinate outside the box.  *out is set only on success. */
srm_status srm_init(const srm_params *p, const double *pos, const double *rho,
                    const double *normals, double s0, int64_t sweep0, int32_t mem_kind,
                    void *stream, srm_ctx **out);

/* One iteration of Algorithm 1's main loop: swell to
 * s' = min(s + c_w*s_target, s_target); up to n_k times bin (Algorithm 2),
 * move every particle (Algorithm 3 over the 2^dim-colour cell schedule) and
 * check for overlaps (Algorithm 6); on the first clean pass commit s'; else
 * discard the swollen copy and shake the committed state (n_k passes at its
 * own radii).  info may be NULL.  Allocates no device memory: every buffer
 * it uses was allocated by srm_init. */
srm_status srm_sweep(srm_ctx *ctx, srm_sweep_info *info);

/* Repeat srm_sweep until the committed volume fraction reaches f_target
 * (Sec. 2 step e: stop at the target fraction).  In these sweeps swelling
 * stops at the scale s_f whose fraction is f_target (to rounding:
 * s_f = (f_target |box| / (w sum_i rho_i^dim))^(1/dim), w = pi for disks,
 * 4 pi/3 for spheres, 2 pi thick_ratio for platelets, 2 pi A^2 h + pi^2 A h^2 +
 * 4/3 pi h^3 with h = thick_ratio, A = 1 - h for spherodisks), or at s_target when
 * that is smaller; f_target <= 0 means s_target itself.  An intermediate
 * target serves staged protocols (grow to f1, change the rates in a new
 * context from the saved state, continue); srm_sweep outside this call
 * always swells toward s_target.  The run ends when the committed scale
 * equals the stop scale.  SRM_ENOTCONV after max_sweeps sweeps; the
 * committed state is then the last admissible one.  SRM_EINVAL if f_target
 * is NaN.  info may be NULL. */
srm_status srm_run_to_fraction(srm_ctx *ctx, double f_target, int32_t max_sweeps,
                               srm_run_info *info);

/* Pairs i < j of the committed state (original ids) whose shapes come within
 * `gap` >= 0 of each other: balls with q_ij <= ((R_i + R_j) + gap)^2 under
 * the minimum image (the hard core - soft shell contact of percolation
 * studies, Sec. 3.3); platelets whose disks, with radii grown to a + gap/2,
 * intersect; spherodisks whose core disks come within h_i + h_j + gap
 * (shells of thickness gap/2 around each surface) (gap = 0: the
 * admissibility test itself).  Written to ij (host
 * or device per mem_kind) as (i, j) int32 pairs sorted by (i, j); *count =
 * number of pairs.  Needs 2 R_max + gap <= min(L_a)/2 (SRM_EINVAL
 * otherwise).  SRM_ECAPACITY (nothing written, *count = the number of
 * pairs) if *count > cap or *count > 2^31 - 1. */
srm_status srm_pairs(srm_ctx *ctx, double gap, int64_t cap, int32_t *ij, int64_t *count,
                     int32_t mem_kind);

/* Histogram of centre distances over pairs i < j of the committed state:
 * pair in bin b = (int)(r_ij * (nbins / r_max)) when b < nbins (r_ij is the
 * correctly rounded sqrt of the minimum-image squared distance).  counts: n
 * bins of uint64 (host).  g (host, nullable): counts normalised by the ideal
 * gas count n(n-1)/2 * shell volume / box volume.  Requires 0 < r_max <=
 * min(L_a)/2 and 1 <= nbins <= 65536. */
srm_status srm_rdf(srm_ctx *ctx, int32_t nbins, double r_max, uint64_t *counts, double *g);

/* Committed state in particle-id order: pos (dim*n), normals (3*n, or NULL),
 * s, sweep (both nullable). */
srm_status srm_get_state(srm_ctx *ctx, double *pos, double *normals, double *s,
                         int64_t *sweep, int32_t mem_kind);

/* Replace the committed positions (and normals, or NULL) with pos (dim*n
 * SoA, id order, every coordinate in [0, L_a)); s and the sweep counter are
 * kept.  Overlaps are allowed: the next srm_sweep resolves them when it
 * commits (with c_w = 0 it only migrates), and reports a shake otherwise.
 * Used after an external update of the positions, e.g. a gradient step. */
srm_status srm_set_state(srm_ctx *ctx, const double *pos, const double *normals,
                         int32_t mem_kind);

/* Release the context and all of its device memory.  NULL is a no-op. */
srm_status srm_free(srm_ctx *ctx);

const char *srm_last_error(void);

/* ---- step-level entry points (parity tests and diagnostics) ---------- */

/* Cells per axis of the adaptive grid for radius scale s (Algorithm 1 cell
 * size: 2.5 * R'max + 2.5 * c_m). */
srm_status srm_grid(srm_ctx *ctx, double s, int32_t na[3]);

/* Cell (linear index cx + Nx*(cy + Ny*cz)) of every committed particle in
 * the grid for radius scale grid_s (Algorithm 2), in id order, host buffer. */
srm_status srm_cells(srm_ctx *ctx, double grid_s, int32_t *cell_by_id);

/* One bin + migration pass (Algorithms 2, 3) on the committed state in
 * place, with the grid for grid_s, radii at scale radius_s, counter fields
 * (kind, k) and the context's current sweep counter; then the global check
 * (Algorithm 6).  acc_by_id (host, nullable): accepted trial per particle
 * (0 = none).  overlap (nullable): 1 if any pair overlaps afterwards. */
srm_status srm_pass(srm_ctx *ctx, double grid_s, double radius_s, int32_t kind, int32_t k,
                    uint8_t *acc_by_id, int32_t *overlap);

/* Accept codes of the last pass run by srm_sweep or srm_pass, id order. */
srm_status srm_last_acc(srm_ctx *ctx, uint8_t *acc_by_id);

/* Nearest-neighbour distances of the committed configuration, the
 * structure descriptor the paper compares its microstructures by (the
 * nearest-neighbour distance distributions of Sec. 3.2, Fig. 4d): for every
 * particle the smallest minimum-image centre distance sqrt(q),
 * q = (d0*d0 + d1*d1) + d2*d2, to another particle with q < r_max^2, or
 * +infinity if there is none (0 < r_max <= L/2).  dist_by_id (host, n
 * doubles, nullable) receives the distances in id order.  hist (host,
 * nbins uint64 counts, nullable; then 1 <= nbins <= 65536) receives the
 * counts of bin (int)(d * (nbins / r_max)) over the particles with a finite
 * d in range.  Balls only.  Errors: SRM_EINVAL. */
srm_status srm_nearest(srm_ctx *ctx, double r_max, double *dist_by_id, int32_t nbins,
                       uint64_t *hist);

/* Hard core - soft shell percolation (the critical percolation distance of
 * Sec. 3.3, Fig. 9): particles are bonded when they overlap after growing
 * by `gap` (the srm_pairs predicate: (R_i + R_j) + gap for balls, disk
 * radii a + gap/2 for platelets, core-disk distance h_i + h_j + gap for
 * spherodisks), and *wraps gets bit a set when a cluster
 * wraps around the periodic box along axis a (a cycle of bonds whose
 * periodic images do not close along a); 0 means no cluster spans the box.
 * Needs 2 R_max + gap <= L/2.  Errors: SRM_EINVAL; SRM_ECAPACITY if a
 * cluster's image offsets exceed +-510 boxes. */
srm_status srm_percolation(srm_ctx *ctx, double gap, int32_t *wraps);
/* Critical percolation distance by bisection on the gap: lo must not
 * percolate and hi must; after `iters` halvings (mid = (lo + hi) / 2, 0 to
 * 200 of them) *gap_c is the final hi, the smallest percolating gap found.
 * Errors: SRM_EINVAL. */
srm_status srm_critical_gap(srm_ctx *ctx, double lo, double hi, int32_t iters, double *gap_c);

/* ---- initial configuration: random sequential addition --------------- */

/* Result counters of srm_rsa. */
typedef struct {
    int64_t drawn;    /* candidates drawn: index of the last one kept + 1, or max_candidates */
    int64_t placed;   /* particles placed (n unless SRM_ENOTCONV) */
    int32_t batches;  /* candidate batches run */
    int32_t rounds;   /* ordering rounds, summed over the batches */
} srm_rsa_info;

/* Classical random sequential addition of n equal particles, the
 * non-overlapping start at a low volume fraction f0 that Sec. 2 and
 * Algorithm 1 begin the swelling from ("RSA procedure").  Candidates
 * k = 0, 1, 2, ... are drawn from Philox4x32-10 keyed by `seed`: the centre
 * from counters (k_lo, k_hi, call, 2) -- per axis a 53-bit uniform
 * ((w_a >> 5) * 2^26 + (w_b >> 6)) * 2^-53 times L_a, words (0,1) and (2,3)
 * of call 0 for x and y, words (0,1) of call 1 for z, a product equal to L_a
 * folded to 0 -- and, for platelets (3D), a unit normal from Algorithm 3's
 * random vector of length 1 with counter (k_lo, k_hi, attempt, 3).  A
 * candidate is kept when it meets no particle kept before it (balls of
 * radius `radius`: minimum-image q <= (radius + radius)^2, touching counts;
 * platelets of radius `radius`: the thin-disk test with the earlier one as
 * disk 1) and gets the next particle id.  The result is that sequence
 * exactly, whatever `batch` (candidates per GPU batch, 0 = automatic, at
 * most 2^28).
 *   pos      dim * n doubles (SoA, id order), written;
 *   normals  3 * n doubles (platelets; NULL for balls), written;
 *   src      n int64 candidate indices (nullable), written;
 *   mem_kind SRM_MEM_HOST or SRM_MEM_DEVICE for these three buffers;
 *   hip_stream the stream all work runs on (NULL = null stream); the call
 *            synchronises it before returning;
 *   info     nullable.
 * Device memory is allocated for the call and freed before it returns.
 * Pass pos/normals with s0 = radius (monodisperse, rho = 1) to srm_init.
 * Errors: SRM_EINVAL (nothing written); SRM_ENOMEM; SRM_ENOTCONV when
 * max_candidates are drawn before n are placed (the first info->placed
 * particles are written). */
srm_status srm_rsa(int32_t dim, int32_t shape, int64_t n, const double *box, double radius,
                   uint64_t seed, int64_t max_candidates, int64_t batch, double *pos,
                   double *normals, int64_t *src, int32_t mem_kind, void *hip_stream,
                   srm_rsa_info *info);

/* ---- differentiable descriptor: soft g(r) + overlap energy -------------- */

/* A workspace for configurations of n particles in a fixed periodic box.
 * Descriptor (steering clustered configurations toward a target radial
 * distribution; SRM's exact test still decides admissibility):
 *   g_b = norm_b * sum_{i<j} K_b(r_ij) w(r_ij),  b < nbins,
 *   K_b(r) = exp(-(r - c_b)^2 / (2 h^2)) / (h sqrt(2 pi)),
 *   c_b = (b + 1/2) D, h = D = r_c / nbins,
 *   w(r) = C2 taper, 1 below r_c, 0 above r_c + 4h,
 *   norm_b = V / (n(n-1)/2 * 4 pi c_b^2)   (2D: 2 pi c_b),
 *   E = kappa/2 * sum_{i<j} max(0, R_i + R_j - r_ij)^2,
 * r_ij the minimum-image distance; FP64 throughout.  Pairs are searched up
 * to r_c + 4h, which must cover every overlapping pair (2 R_max <= r_c +
 * 4h).  Every buffer below is device memory; all work runs on `stream`;
 * results are deterministic (fixed-order reductions, no atomics). */
typedef struct {
    int32_t dim;      /* 2 or 3 */
    int32_t nbins;    /* 1 .. 64 */
    double box[3];    /* periodic box edges */
    double r_c;       /* bins cover [0, r_c] */
    double kappa;     /* penalty stiffness */
} srm_softrdf_params;

typedef struct srm_soft srm_soft;

srm_status srm_softrdf_create(const srm_softrdf_params *p, int64_t n, void *stream,
                              srm_soft **out);
/* pos: dim*n SoA in [0, L_a); radii: n.  g_out: nbins; energy: 1 double. */
srm_status srm_softrdf_forward(srm_soft *ctx, const double *pos, const double *radii,
                               double *g_out, double *energy);
/* dg: dL/dg (nbins); dE: dL/dE (1 double).  grad_pos: dim*n SoA;
 * grad_radii: n.  Pairs are recomputed from pos, not stored. */
srm_status srm_softrdf_backward(srm_soft *ctx, const double *pos, const double *radii,
                                const double *dg, const double *dE, double *grad_pos,
                                double *grad_radii);
srm_status srm_softrdf_free(srm_soft *ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or steering loops, harnesses that forbid
 * hipMalloc): the forward above without a workspace.  Same definitions,
 * kernels and arguments as srm_softrdf_create + srm_softrdf_forward (the
 * results are bit-identical), but the working memory (cell-sorted copies,
 * binning scratch, block partials) is a fixed device array inside the
 * library, ~17 MB, which every device the library runs on holds until the
 * process ends.  Allocates nothing: no hipMalloc, hipFree or allocating
 * library call.  pos (dim*n SoA), radii (n), g_out (nbins) and energy (1)
 * are device memory owned by the caller; pos and radii are only read.
 * n must be 2 .. SRM_SOFTRDF_STATIC_MAX_N, else SRM_ECAPACITY (beyond the
 * limit) or SRM_EINVAL, with nothing launched.  Every call on one device
 * shares that device's array: calls that overlap in time on one device
 * (two streams, two threads) race and give undefined results; calls in
 * one stream are ordered and safe. */
#define SRM_SOFTRDF_STATIC_MAX_N 262144
srm_status srm_softrdf_forward_static(const srm_softrdf_params *p, int64_t n,
                                      const double *pos, const double *radii, double *g_out,
                                      double *energy, void *stream);

/* ---- batched ensembles ------------------------------------------------- */

/* `count` independent periodic boxes (RVEs) of balls, 2D and 3D mixed, each
 * with its own srm_params (shape SRM_BALL, n_k >= 1), advanced together:
 * the per-RVE Algorithm 1 state lives on the device and a captured hipGraph
 * of batched kernels moves every unfinished RVE by a few passes per replay.
 * pos: the RVEs' dim*n SoA blocks one after another (host); rho: their n
 * shape radii one after another (host), or NULL for all 1.  All RVEs start
 * at s = 0 with sweep counter 0.  Each RVE's result is bit-identical to
 * srm_run_to_fraction on the same inputs. */
typedef struct srm_batch srm_batch;

typedef struct {
    int64_t replays;        /* graph replays of this run (up to 3 queued after the last
                               RVE finished, which change nothing) */
    int64_t slots;          /* pass slots (replays * slots per replay) */
    int32_t converged;      /* RVEs at their target */
    int32_t not_converged;  /* RVEs that used up max_sweeps */
    int64_t passes;         /* migration passes summed over RVEs */
    int64_t updates;        /* particle updates summed over RVEs */
} srm_batch_info;

srm_status srm_batch_init(int32_t count, const srm_params *params, const double *pos,
                          const double *rho, srm_batch **out);
/* Schedule only (results do not depend on it): pass slots per graph replay
 * (1..64), threads per block of the sparse-grid migration kernels (64, 128
 * or 256; a group of lanes shares a cell there), and the mean particles per
 * cell (1..64, default 3) from which an RVE's grid migrates with one
 * wavefront per cell instead. */
srm_status srm_batch_configure(srm_batch *b, int32_t slots_per_replay, int32_t block,
                               int32_t wave_occupancy);
/* Run until every RVE converged or used max_sweeps more sweeps
 * (SRM_ENOTCONV then; converged RVEs keep their result).  Replays are
 * queued four ahead of the host's check of the unfinished count, so the
 * device does not wait on the host between replays. */
srm_status srm_batch_run(srm_batch *b, int32_t max_sweeps, srm_batch_info *info);
/* Committed state of RVE r: pos (dim*n, host, id order), s, sweep counter,
 * passes run so far (all nullable). */
srm_status srm_batch_get(srm_batch *b, int32_t r, double *pos, double *s, int64_t *sweep,
                         int64_t *passes);
srm_status srm_batch_free(srm_batch *b);
const char *srm_batch_last_error(void);

/* ---- device-time profile ------------------------------------------------ */

/* Device time of the sweep's kernels, measured with hipEvents recorded on
 * the context's stream around each binning run (Algorithm 2), each colour
 * phase of a migration pass (Algorithm 3) and each global check
 * (Algorithm 6).  Milliseconds accumulate from the last srm_profile_enable. */
typedef struct {
    double ms_bin, ms_migrate, ms_check;
    int64_t bins;              /* binning runs */
    int64_t launches_migrate;  /* colour-phase launches */
    int64_t passes;            /* migration passes */
    int64_t checks;            /* global checks */
    double ms_migrate_main;    /* the colour phases' main kernels alone (no overflow launch) */
    int64_t main_kernels;      /* SRM_KERNEL_* bits of the main kernels that ran */
    int64_t trials;            /* trial moves of every pass while counting is on: the
                                  accepted trial's index, or N_l for a rejection */
} srm_profile;

/* Main migration kernel of a colour phase (srm_profile.main_kernels). */
#define SRM_KERNEL_TILE 1     /* LDS-tiled, four lanes per cell */
#define SRM_KERNEL_WAVE 2     /* one wavefront per cell (crowded or small grids) */
#define SRM_KERNEL_CELL 4     /* reserved: one thread per cell (not selected) */
#define SRM_KERNEL_PLATELET 8 /* platelets (with SRM_KERNEL_WAVE) */
#define SRM_KERNEL_TILE_WIDE 16 /* LDS-tiled with the largest region (denser 3D grids) */
#define SRM_KERNEL_TILE_MID 32  /* LDS-tiled with a middle region (3D) */

/* Profiling switches, reset with the accumulated profile: bit 0 times the
 * phases above with hipEvents; bit 1 also counts trial moves (a small
 * reduction over the accept codes after every pass, so it adds work). */
srm_status srm_profile_enable(srm_ctx *ctx, int32_t on);
/* Copy the accumulated profile (synchronises the stream). */
srm_status srm_profile_read(srm_ctx *ctx, srm_profile *out);

/* ---- diagnostics of the device arithmetic ------------------------------ */

/* Device results, for host arrays of n inputs, of IEEE binary64 sqrt(a[i])
 * and a[i] / b[i] as the kernels compute them (the bit-exact contract needs
 * both correctly rounded).  n >= 0; all buffers host memory. */
srm_status srm_debug_fp(const double *a, const double *b, int64_t n, double *sqrt_out,
                        double *div_out);

/* Philox4x32-10 on the device: out[4i..4i+3] = philox(ctr[4i..4i+3],
 * key[2i..2i+1]) for i < n.  Host buffers. */
srm_status srm_debug_philox(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out);

/* The trial-move random vector (length len, dim 2 or 3) drawn on the device
 * for particle ids 0..n-1 with sweep t and counter word
 * word = kind<<31 | k<<16 | l<<8: out[3i..3i+2] (z = 0 in 2D).  Host
 * buffer. */
srm_status srm_debug_unitvec(int32_t dim, uint64_t seed, uint32_t t, uint32_t word,
                             uint32_t stream, double len, int64_t n, double *out);

#ifdef __cplusplus
}
#endif

#endif /* SRM_H */
