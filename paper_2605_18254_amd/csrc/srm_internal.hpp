// srm_internal.hpp -- context layout and the host launchers shared by the
// translation units of libsrm (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "srm.h"
#include "srm_device.hpp"

namespace srm {

// Particle arrays of one storage order (cells ascending, ids ascending
// within a cell after a rebin).  Unused arrays are null.
struct PBuf {
    double *x[3];
    double *nrm[3];
    double *rho;
    int32_t *id;
};

// Small device-side result block of the global check.
struct Counters {
    int32_t overlap;     // 1 if a colliding particle was found
    int32_t bad;         // 1 if an input coordinate was outside the box
    int64_t unused;      // keeps the layout
    int32_t nfail_list;  // host copy of the failed-list length
    int32_t pad;
};

struct Scratch {
    int32_t *cell;      // [n] destination cell per source slot
    int32_t *slot;      // [n] rank within the destination cell (atomic order)
    int32_t *tmpid;     // [n] ids in arrival order, for the in-cell ranks
    int32_t *counts;    // [cap] particles per cell
    int32_t *start;     // [cap + 1] exclusive prefix of counts
    int32_t *partials;  // per-block sums of the scan
    int64_t cap;        // cell capacity (>= every grid's ncell)
};

// Launch configuration of one migration colour phase.
struct ColourLattice {
    int32_t h[3];   // colour cells per axis
    int32_t off[3]; // parity offset per axis
    int32_t count;  // colour cells in this phase
};

// Sets the message srm_last_error() returns (thread-local).
void set_last_error(const char *msg);

// Host launchers (all enqueue on `stream`).
hipError_t launch_fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t stream);
hipError_t launch_fill_u8(uint8_t *a, int64_t n, uint8_t v, hipStream_t stream);
hipError_t launch_zero_counters(Counters *c, hipStream_t stream);
// *total += sum over slots of (acc ? acc : n_l): the trials a pass ran.
hipError_t count_trials(const uint8_t *acc, int32_t n, int32_t n_l,
                        unsigned long long *total, hipStream_t stream);
hipError_t launch_iota(int32_t *a, int32_t n, hipStream_t stream);
// *total = a[0] + ... + a[n-1] in 64 bits (zeroed first; a[i] >= 0).
hipError_t sum_counts64(const int32_t *a, int32_t n, unsigned long long *total,
                        hipStream_t stream);

// Counting sort of `src` by the cells of `g` into `dst` (Algorithm 2's
// lists as a cell-sorted CSR array `sc.start`, ids ascending within a cell).
hipError_t bin_particles(int dim, const PBuf &src, const PBuf &dst, int32_t n, const Grid &g,
                         Scratch &sc, Counters *cnt, hipStream_t stream);
// Exclusive scan of counts[0..m) into start[0..m] (start[m] = total).
hipError_t scan_counts(const int32_t *counts, int32_t *start, int32_t *partials, int32_t m,
                       hipStream_t stream);
// Scatter sorted-order arrays to particle-id order: out[a*n + id[p]] = x[a][p].
hipError_t to_id_order(const double *const *x, int nx, const int32_t *id, int32_t n, double *out,
                       hipStream_t stream);
hipError_t u8_to_id_order(const uint8_t *a, const int32_t *id, int32_t n, uint8_t *out,
                          hipStream_t stream);
hipError_t cells_by_id(int dim, const PBuf &b, int32_t n, const Grid &g, int32_t *out,
                       hipStream_t stream);

struct PassArgs {
    PBuf buf;
    const int32_t *start;
    uint8_t *acc;
    Grid g;
    int32_t n;
    double s;          // radius scale of this pass
    double sig2_mono;  // (s + s)^2 for monodisperse balls
    Draw draw;         // key, sweep, kind<<31 | k<<16 (trial l added per draw)
    int32_t n_l;
    double c_m, c_n;
    double tau;            // platelets: half-thickness / outer radius (0: zero-thickness disks)
    int32_t *ovf;          // tiled kernel: per-colour overflow counts + tile lists
    int32_t ovf_max_tiles; // list capacity per colour
    int32_t *failed;       // [0] = count, then slots of particles that rejected every trial
};

// One colour phase of a migration pass (Algorithm 3 over the cells whose
// parity vector is `colour`); *launched is false for an empty phase.
// One colour phase of Algorithm 3.  If `after_main` is given it is recorded
// right after the phase's main kernel (before any overflow launch), and
// *which gets that kernel's kind (SRM_KERNEL_* bits of srm_profile).
hipError_t migrate_colour(int dim, int shape, bool poly, const PassArgs &a, int colour,
                          hipStream_t stream, bool *launched, hipEvent_t after_main = nullptr,
                          int *which = nullptr);
// Global check (Algorithm 6) restricted to particles with accept code 0
// (or every particle when check_all), result into cnt.
hipError_t check_overlaps(int dim, int shape, bool poly, const PassArgs &a, bool check_all,
                          Counters *cnt, hipStream_t stream);

// Pair enumeration and distance histogram of a binned configuration
// (k_pairs.hip).  rowcnt/rowoff are indexed by particle id.
hipError_t pairs_count(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                       int shape, double tau, double s, double gap, int32_t *rowcnt,
                       hipStream_t stream);
hipError_t pairs_emit(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                      int shape, double tau, double s, double gap, const int32_t *rowoff,
                      int32_t *partner, int32_t *ij, hipStream_t stream);
hipError_t rdf_counts(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                      int32_t nbins, double inv, unsigned long long *counts, hipStream_t stream);
// Percolation (k_perc.hip): bond image shifts, (label, offset) relaxation
// until flags[0] stays 0 (flags[1]: offset overflow), then the wrapping axes
// OR-ed into flags[2].
hipError_t bond_shifts(const int32_t *ij, int64_t nb, const double *pos_by_id, int32_t n, int dim,
                       const Grid &g, int32_t *shift, hipStream_t stream);
hipError_t perc_init(unsigned long long *state, int32_t n, hipStream_t stream);
hipError_t perc_relax(const int32_t *ij, const int32_t *shift, int64_t nb,
                      unsigned long long *state, int32_t *flags, hipStream_t stream);
hipError_t perc_check(const int32_t *ij, const int32_t *shift, int64_t nb,
                      const unsigned long long *state, int32_t *flags, hipStream_t stream);
// Nearest-neighbour distance (by id, nullable) and its histogram (nullable)
// for every particle, searched within r_max (grid cells >= r_max).
hipError_t nearest(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                   double r_max, double *dist, int32_t nbins, unsigned long long *counts,
                   hipStream_t stream);

// Soft-binned g(r) + overlap energy and its gradient (k_softrdf.hip).
// Soft g(r) launch shape: threads per block of the forward kernel and
// doubles per block partial (64 bins, then the energy).
constexpr int32_t kSoftBlock = 128;
constexpr int32_t kSoftPartialStride = 65;
int32_t soft_blocks(int32_t n);
int32_t soft_partial_stride();
hipError_t soft_forward(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                        int32_t nbins, double r_c, double kappa, double *partial, double *gout,
                        double *energy, hipStream_t stream);
hipError_t soft_backward(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                         int32_t nbins, double r_c, double kappa, const double *dg,
                         const double *dE, double *gpos, double *grad_r, hipStream_t stream);

// Diagnostics of the device arithmetic (k_diag.hip).
hipError_t diag_fp(const double *a, const double *b, int32_t n, double *sq, double *dv,
                   hipStream_t s);
hipError_t diag_philox(const uint32_t *ctr, const uint32_t *key, int32_t n, uint32_t *out,
                       hipStream_t s);
hipError_t diag_unitvec(int dim, uint64_t seed, uint32_t t, uint32_t word, uint32_t stream,
                        double len, int32_t n, double *out, hipStream_t s);

}  // namespace srm
