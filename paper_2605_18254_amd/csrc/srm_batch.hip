// srm_batch.hip -- a whole ensemble of independent periodic boxes (RVEs) of
// uneven sizes, dimensions and targets, advanced together on one GPU.
//
// Each RVE keeps its own Algorithm 1 state on the device (radius scale,
// sweep counter, current pass, which buffer holds P, Q, T) in a small
// control record, so the sweep logic that srm_sweep runs on the host runs
// here in a control kernel, one thread per RVE.  One "pass slot" is a fixed
// sequence of batched kernels:
//   control (swell / grid / pass selection) -> counting sort of every active
//   RVE at once -> 2^dim colour launches per dimension class -> check of the
//   failed particles -> control (commit, next pass, shake, next sweep).
// RVEs that finished their sweep, converged or ran out of sweeps idle.  A
// run captures K pass slots in one hipGraph and replays it until no RVE is
// left, so the host only polls one counter per replay.  Every RVE runs
// exactly the operations of its solo run (same grid, order, counters,
// decisions), so its result is bit-identical to srm_run_to_fraction.
//
// Layout: all RVEs' particles are concatenated (RVE r at [off_r,
// off_r + n_r)) in three buffer sets; cell slots are concatenated with
// capacity n_r + 2 per RVE, so one global scan of the counts yields global
// particle offsets (an idle RVE parks its n_r particles in its last slot).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "srm_cellpass.hpp"

namespace srm {
namespace {

constexpr int kB = 256;
// Lanes per colour cell of a sparse-grid launch, and cells per wavefront
// (the fastest of 2 to 16 lanes in 3D and of 1 to 8 in 2D, timed on the
// 256-RVE ensemble).
template <int DIM>
struct Sparse {
    static constexpr int kGroup = (DIM == 3) ? 4 : 2;
    static constexpr int kCells = 64 / kGroup;
    static_assert(64 % kGroup == 0, "a group stays inside one wavefront");
};
constexpr int32_t kWaveGrid = 8192;  // workgroups of a wavefront-per-cell launch

enum : int32_t { kSweepStart = 0, kMain = 1, kShake = 2, kDone = 3, kNotConv = 4 };
enum : int32_t { kRoleP = 0, kRoleQ = 1, kRoleT = 2 };

struct Rve {
    // fixed
    int32_t dim, n, off, coff;
    int32_t n_k, n_l, poly, pad0;
    double box[3];
    double s_target, c_w, c_m, rho_max;
    uint32_t key0, key1;
    int64_t ncap;
    // dynamic
    double s, s1, pass_s;
    int64_t t;
    int32_t mode, k, sweeps, passes, shakes, max_sweeps;
    int32_t role[3];
    int32_t active, src, dst, kind;
    int32_t overlap, wave;  // wave: crowded grid, one wavefront per cell
    Grid g;
    int32_t ccount[8];
};

struct BatchDev {
    Rve *rve;
    int32_t count;
    int32_t ntotal;        // sum of n_r
    int32_t ncells;        // sum of (n_r + 2)
    int32_t pad;
    double *x[3][3];       // [set][axis]
    int32_t *id[3];
    double *rho[3];
    int32_t *rve_of;       // particle slot -> RVE
    int32_t *rve_of_cell;  // cell slot -> RVE
    int32_t *cell, *slot, *counts, *start, *partials;
    int32_t *tmpid;        // ids scattered in arrival order, for the in-cell ranks
    uint8_t *acc;
    int32_t *failed;       // [0] count, then global slots
    int32_t *prefix;       // [4 classes (dim, wave)][8 colours][count + 1]
    int32_t *remaining;
    int32_t wave_occ;      // mean particles per cell from which a grid is crowded
};

__device__ __forceinline__ PBuf set_buf(const BatchDev &d, int set)
{
    PBuf b{};
    b.x[0] = d.x[set][0];
    b.x[1] = d.x[set][1];
    b.x[2] = d.x[set][2];
    b.id = d.id[set];
    b.rho = d.rho[set];
    return b;
}

__device__ __forceinline__ PassArgs pass_args_of(const BatchDev &d, const Rve &r)
{
    PassArgs a{};
    a.buf = set_buf(d, r.dst);
    if (!r.poly) a.buf.rho = nullptr;
    a.start = d.start + r.coff;
    a.acc = d.acc;
    a.g = r.g;
    a.n = r.n;
    a.s = r.pass_s;
    const double sig = r.pass_s + r.pass_s;
    a.sig2_mono = sig * sig;
    a.draw.key0 = r.key0;
    a.draw.key1 = r.key1;
    a.draw.t = (uint32_t)r.t;
    a.draw.word = counter_word((uint32_t)r.kind, (uint32_t)r.k, 0);
    a.n_l = r.n_l;
    a.c_m = r.c_m;
    a.failed = d.failed;
    return a;
}

// ---- control ------------------------------------------------------------

__global__ void k_ctl_begin(BatchDev d)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    Rve &r = d.rve[i];
    r.active = 0;
    r.overlap = 0;
    if (r.mode == kDone || r.mode == kNotConv) return;
    if (r.mode == kSweepStart) {
        if (!(r.s < r.s_target)) {
            r.mode = kDone;
            return;
        }
        if (r.sweeps >= r.max_sweeps) {
            r.mode = kNotConv;
            return;
        }
        r.s1 = swell_scale(r.s, r.c_w, r.s_target);
        r.g = sweep_grid(r.dim, r.box, r.ncap, r.c_m, r.s1 * r.rho_max);
        for (int c = 0; c < 8; ++c) {
            int32_t cnt = 1;
            for (int ax = 0; ax < 3; ++ax) {
                const int bit = (c >> ax) & 1;
                if (ax < r.dim && r.g.na[ax] >= 4) cnt *= r.g.na[ax] / 2;
                else if (bit) cnt = 0;
            }
            r.ccount[c] = (c < (1 << r.dim)) ? cnt : 0;
        }
        int64_t ncell = 1;
        for (int ax = 0; ax < r.dim; ++ax) ncell *= r.g.na[ax];
        r.wave = (int64_t)r.n >= (int64_t)d.wave_occ * ncell;
        r.mode = kMain;
        r.k = 1;
    }
    if (r.mode == kMain) {
        r.kind = SRM_PASS_MAIN;
        r.pass_s = r.s1;
        if (r.k == 1) {
            r.src = r.role[kRoleP];
            r.dst = r.role[kRoleQ];
        } else {
            r.src = r.role[kRoleQ];
            r.dst = r.role[kRoleT];
            r.role[kRoleT] = r.role[kRoleQ];
            r.role[kRoleQ] = r.dst;
        }
    } else {  // shake: P re-binned into T, which becomes P
        r.kind = SRM_PASS_SHAKE;
        r.pass_s = r.s;
        r.src = r.role[kRoleP];
        r.dst = r.role[kRoleT];
        r.role[kRoleT] = r.role[kRoleP];
        r.role[kRoleP] = r.dst;
    }
    r.active = 1;
}

// Exclusive prefix over the RVEs of their work units, one list per (class,
// colour) j = class * 8 + colour (class: 2D/3D x sparse/crowded grid),
// counting only active RVEs of that class.  A crowded grid's unit is a
// colour cell (one wavefront each), a sparse grid's a wavefront's worth of
// Sparse<dim>::kCells colour cells.  One thread per RVE, 256 RVEs a chunk, a
// wavefront scan per list.
constexpr int kCtlBlock = 256;

__global__ void __launch_bounds__(kCtlBlock) k_ctl_prefix(BatchDev d)
{
    __shared__ int32_t wtot[32][kCtlBlock / 64];
    __shared__ int32_t carry[32];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < 32) carry[tid] = 0;
    __syncthreads();
    for (int32_t base = 0; base < d.count; base += kCtlBlock) {
        const int32_t i = base + tid;
        bool act = false;
        int32_t dim = 0, wave = 0, cc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) cc[c] = 0;
        if (i < d.count) {
            const Rve &r = d.rve[i];
            act = r.active != 0;
            dim = r.dim;
            wave = r.wave;
#pragma unroll
            for (int c = 0; c < 8; ++c) cc[c] = r.ccount[c];
        }
        int32_t v[32], incl[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const int cls = j >> 3;
            const bool m = act && dim == ((cls >> 1) ? 3 : 2) && wave == (cls & 1);
            // sparse-grid classes count wavefronts of Sparse<dim>::kCells cells
            const int cpw = (cls >> 1) ? Sparse<3>::kCells : Sparse<2>::kCells;
            v[j] = !m ? 0 : (cls & 1) ? cc[j & 7] : (cc[j & 7] + cpw - 1) / cpw;
            int32_t x = v[j];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t u = __shfl_up(x, o, 64);
                if (lane >= o) x += u;
            }
            incl[j] = x;
        }
        if (lane == 63)
#pragma unroll
            for (int j = 0; j < 32; ++j) wtot[j][wv] = incl[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            int32_t off = carry[j];
            for (int w = 0; w < wv; ++w) off += wtot[j][w];
            if (i < d.count) d.prefix[(size_t)j * (d.count + 1) + i] = off + incl[j] - v[j];
        }
        __syncthreads();
        if (tid < 32) {
            int32_t t = 0;
            for (int w = 0; w < kCtlBlock / 64; ++w) t += wtot[tid][w];
            carry[tid] += t;
        }
        __syncthreads();
    }
    if (tid < 32) d.prefix[(size_t)tid * (d.count + 1) + d.count] = carry[tid];
}

__global__ void k_ctl_end(BatchDev d)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    Rve &r = d.rve[i];
    if (!r.active) return;
    r.passes += 1;
    if (r.mode == kMain) {
        if (!r.overlap) {
            const int32_t p = r.role[kRoleP];
            r.role[kRoleP] = r.role[kRoleQ];
            r.role[kRoleQ] = p;
            r.s = r.s1;
            r.t += 1;
            r.sweeps += 1;
            r.mode = kSweepStart;
        } else if (r.k < r.n_k) {
            r.k += 1;
        } else {
            r.mode = kShake;
            r.k = 1;
        }
    } else {
        if (r.k < r.n_k) {
            r.k += 1;
        } else {
            r.t += 1;
            r.sweeps += 1;
            r.shakes += 1;
            r.mode = kSweepStart;
        }
    }
}

__global__ void k_count_remaining(BatchDev d)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.count) return;
    const Rve &r = d.rve[i];
    const bool left = !(r.mode == kDone || r.mode == kNotConv ||
                        (r.mode == kSweepStart && !(r.s < r.s_target)));
    if (left) atomicAdd(d.remaining, 1);
}

__global__ void k_zero1(int32_t *p)
{
    if (threadIdx.x == 0) *p = 0;
}

// ---- batched counting sort -------------------------------------------------

__global__ void __launch_bounds__(kB) k_bfill(BatchDev d)
{
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells) return;
    const Rve &r = d.rve[d.rve_of_cell[c]];
    const int32_t local = c - r.coff;
    d.counts[c] = (!r.active && local == r.n + 1) ? r.n : 0;
}

__global__ void __launch_bounds__(kB) k_bcount(BatchDev d)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t key = -1;
    bool live = false;
    if (p < d.ntotal) {
        const Rve &r = d.rve[d.rve_of[p]];
        if (r.active) {
            live = true;
            const int s = r.src;
            const double px = d.x[s][0][p], py = d.x[s][1][p];
            const double pz = (r.dim == 3) ? d.x[s][2][p] : 0.0;
            const int32_t c = (r.dim == 3) ? cell_of<3>(r.g, px, py, pz)
                                           : cell_of<2>(r.g, px, py, pz);
            key = r.coff + c;
        }
    }
    // one atomic per run of equal cell slots in the wavefront
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(key, 1, 64);
    const bool head = live && (lane == 0 || prev != key);
    const unsigned long long heads = __ballot(head);
    const unsigned long long lv = __ballot(live);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const unsigned long long below = heads & upto;
    const int first = below ? 63 - __clzll(below) : lane;
    const unsigned long long above = heads & ~upto;
    int next = above ? __ffsll((long long)above) - 1 : 64;
    // a run ends at the next head or at the first dead lane after it
    const unsigned long long dead_above = ~lv & ~upto;
    const int next_dead = dead_above ? __ffsll((long long)dead_above) - 1 : 64;
    if (next_dead < next) next = next_dead;
    int32_t base = 0;
    if (head) base = atomicAdd(&d.counts[key], next - lane);
    base = __shfl(base, first, 64);
    if (!live) return;
    d.cell[p] = key;
    d.slot[p] = base + (lane - first);
}

// Counting-sort placement without a sort pass: ids go to their cells in
// arrival order first, then every particle counts the smaller ids of its
// cell -- its rank in ascending id order -- and moves its record there.
__global__ void __launch_bounds__(kB) k_bscatter_id(BatchDev d)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.ntotal) return;
    const Rve &r = d.rve[d.rve_of[p]];
    if (!r.active) return;
    d.tmpid[d.start[d.cell[p]] + d.slot[p]] = d.id[r.src][p];
}

__global__ void __launch_bounds__(kB) k_brank(BatchDev d)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.ntotal) return;
    const Rve &r = d.rve[d.rve_of[p]];
    if (!r.active) return;
    const int s = r.src, t = r.dst;
    const int32_t c = d.cell[p];
    const int32_t b = d.start[c], e = d.start[c + 1];
    const int32_t me = d.id[s][p];
    int32_t rank = 0;
    for (int32_t q = b; q < e; ++q) rank += d.tmpid[q] < me;
    const int32_t q = b + rank;
    d.x[t][0][q] = d.x[s][0][p];
    d.x[t][1][q] = d.x[s][1][p];
    if (r.dim == 3) d.x[t][2][q] = d.x[s][2][p];
    d.id[t][q] = me;
    if (r.poly) d.rho[t][q] = d.rho[s][p];
}

// Sparse<DIM>::kGroup lanes per colour cell of every active RVE of
// dimension DIM whose grid is sparse; a wavefront takes Sparse<DIM>::kCells
// cells of one RVE, so the RVE's record is read once per wavefront.  The
// group runs Algorithm 3 for its cell with the trial's stencil split over
// its lanes (migrate_cell_lanes).
template <int DIM, bool POLY>
__global__ void __launch_bounds__(kB) k_bmigrate(BatchDev d, int colour)
{
    constexpr int kGroup = Sparse<DIM>::kGroup;
    const int32_t *pre = d.prefix + (size_t)((DIM == 3 ? 16 : 0) + colour) * (d.count + 1);
    const int32_t w = __builtin_amdgcn_readfirstlane((int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int lane = threadIdx.x & 63;
    if (w >= pre[d.count]) return;  // wavefront-uniform
    int32_t lo = 0, hi = d.count - 1;  // last RVE with pre[i] <= w
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    const Rve &r = d.rve[lo];
    const int32_t u = (w - pre[lo]) * Sparse<DIM>::kCells + lane / kGroup;
    if (u >= r.ccount[colour]) return;  // group-uniform
    int32_t h[3], off[3];
    for (int ax = 0; ax < 3; ++ax) {
        const bool split = ax < DIM && r.g.na[ax] >= 4;
        h[ax] = split ? r.g.na[ax] / 2 : 1;
        off[ax] = split ? (colour >> ax) & 1 : 0;
    }
    const int32_t jx = u % h[0], jy = (u / h[0]) % h[1], jz = u / (h[0] * h[1]);
    const PassArgs a = pass_args_of(d, r);
    migrate_cell_lanes<DIM, POLY, kGroup>(a, 2 * jx + off[0], 2 * jy + off[1],
                                          (DIM == 3) ? 2 * jz + off[2] : 0);
}

// One 64-thread workgroup per colour cell of every active RVE of dimension
// DIM whose grid is crowded (grid-stride over those cells).
template <int DIM, bool POLY>
__global__ void __launch_bounds__(64) k_bmigrate_wave(BatchDev d, int colour)
{
    __shared__ WaveLds lds;
    const int32_t *pre = d.prefix + (size_t)((DIM == 3 ? 24 : 8) + colour) * (d.count + 1);
    const int32_t total = pre[d.count];
    for (int32_t t = blockIdx.x; t < total; t += gridDim.x) {
        int32_t lo = 0, hi = d.count - 1;  // last RVE with pre[i] <= t
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const Rve &r = d.rve[lo];
        const int32_t u = t - pre[lo];
        int32_t h[3], off[3];
        for (int ax = 0; ax < 3; ++ax) {
            const bool split = ax < DIM && r.g.na[ax] >= 4;
            h[ax] = split ? r.g.na[ax] / 2 : 1;
            off[ax] = split ? (colour >> ax) & 1 : 0;
        }
        const int32_t jx = u % h[0], jy = (u / h[0]) % h[1], jz = u / (h[0] * h[1]);
        const PassArgs a = pass_args_of(d, r);
        migrate_cell_wave<DIM, POLY>(a, 2 * jx + off[0], 2 * jy + off[1],
                                     (DIM == 3) ? 2 * jz + off[2] : 0, lds);
        __syncthreads();  // LDS is reused by the next cell
    }
}

// One wavefront per failed particle (grid-stride over the failed list).
template <bool POLY>
__global__ void __launch_bounds__(kB) k_bcheck(BatchDev d)
{
    const int32_t count = d.failed[0];
    const int lane = threadIdx.x & 63;
    const int32_t waves = gridDim.x * (kB / 64);
    for (int32_t i = blockIdx.x * (kB / 64) + (threadIdx.x >> 6); i < count; i += waves) {
        const int32_t p = d.failed[1 + i];
        Rve &r = d.rve[d.rve_of[p]];
        if (__atomic_load_n(&r.overlap, __ATOMIC_RELAXED)) continue;  // already known
        const PassArgs a = pass_args_of(d, r);
        const bool hit = (r.dim == 3) ? check_ball_wave<3, POLY>(a, p, lane)
                                      : check_ball_wave<2, POLY>(a, p, lane);
        if (hit && lane == 0) atomicOr(&r.overlap, 1);
    }
}

inline unsigned nblk(int64_t n, int b = kB)
{
    const int64_t x = (n + b - 1) / b;
    return (unsigned)(x > 0 ? x : 1);
}

}  // namespace

// Graph replays kept in flight by srm_batch_run.
constexpr int kDepth = 4;

// Host-side record of a batch (opaque through the C ABI).
struct BatchHost {
    BatchDev d{};
    std::vector<Rve> init;     // initial control records (for reruns)
    hipStream_t stream = nullptr;
    bool poly = false;
    int32_t bound[2] = {0, 0};  // colour-cell bound per dimension class
    int32_t slots = 4;          // pass slots per graph replay
    int32_t block = kB;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *hrem = nullptr;    // pinned, one count per replay in flight
    hipEvent_t done[kDepth] = {};  // recorded after each replay's count copy
    std::vector<void *> allocs;
};

}  // namespace srm

using namespace srm;

namespace {

thread_local std::string g_batch_error;

srm_status bfail(srm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
srm_status bfail(srm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_batch_error = buf;
    return st;
}

#define BHIP(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return bfail(SRM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

template <class T_>
hipError_t balloc(BatchHost *h, T_ **ptr, size_t count)
{
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, (count > 0 ? count : 1) * sizeof(T_));
    if (e == hipSuccess) {
        h->allocs.push_back(v);
        *ptr = (T_ *)v;
    }
    return e;
}

// One pass slot of the batched sweep (all launches on h->stream).
hipError_t enqueue_slot(BatchHost *h)
{
    BatchDev &d = h->d;
    hipStream_t s = h->stream;
    const unsigned rb = nblk(d.count, 64);
    hipLaunchKernelGGL(k_ctl_begin, dim3(rb), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_ctl_prefix, dim3(1), dim3(kCtlBlock), 0, s, d);
    // Algorithm 2 for every active RVE: counting sort src -> dst
    hipLaunchKernelGGL(k_bfill, dim3(nblk(d.ncells)), dim3(kB), 0, s, d);
    hipLaunchKernelGGL(k_bcount, dim3(nblk(d.ntotal)), dim3(kB), 0, s, d);
    hipError_t e = scan_counts(d.counts, d.start, d.partials, d.ncells, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bscatter_id, dim3(nblk(d.ntotal)), dim3(kB), 0, s, d);
    hipLaunchKernelGGL(k_brank, dim3(nblk(d.ntotal)), dim3(kB), 0, s, d);
    // Algorithm 3 over the colour schedule, per dimension class
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, s, d.failed);
    for (int dc = 0; dc < 2; ++dc) {
        const int dim = dc ? 3 : 2;
        if (h->bound[dc] == 0) continue;
        // sparse grids: at most ccount / kCells + 1 wavefronts an RVE
        const int64_t waves = h->bound[dc] / (dc ? Sparse<3>::kCells : Sparse<2>::kCells) + d.count;
        const dim3 grid(nblk(waves * 64, h->block)), block(h->block);
        const dim3 wgrid(h->bound[dc] < kWaveGrid ? h->bound[dc] : kWaveGrid), wblock(64);
        for (int colour = 0; colour < (1 << dim); ++colour) {
            // sparse grids: a lane group per cell; crowded grids: a wavefront per cell
            if (dim == 3) {
                if (h->poly) {
                    hipLaunchKernelGGL((k_bmigrate<3, true>), grid, block, 0, s, d, colour);
                    hipLaunchKernelGGL((k_bmigrate_wave<3, true>), wgrid, wblock, 0, s, d, colour);
                } else {
                    hipLaunchKernelGGL((k_bmigrate<3, false>), grid, block, 0, s, d, colour);
                    hipLaunchKernelGGL((k_bmigrate_wave<3, false>), wgrid, wblock, 0, s, d, colour);
                }
            } else {
                if (h->poly) {
                    hipLaunchKernelGGL((k_bmigrate<2, true>), grid, block, 0, s, d, colour);
                    hipLaunchKernelGGL((k_bmigrate_wave<2, true>), wgrid, wblock, 0, s, d, colour);
                } else {
                    hipLaunchKernelGGL((k_bmigrate<2, false>), grid, block, 0, s, d, colour);
                    hipLaunchKernelGGL((k_bmigrate_wave<2, false>), wgrid, wblock, 0, s, d, colour);
                }
            }
        }
    }
    // Algorithm 6 on the particles that rejected every trial
    const unsigned cb = nblk(d.ntotal) < 1024 ? nblk(d.ntotal) : 1024;
    if (h->poly) hipLaunchKernelGGL(k_bcheck<true>, dim3(cb), dim3(kB), 0, s, d);
    else hipLaunchKernelGGL(k_bcheck<false>, dim3(cb), dim3(kB), 0, s, d);
    hipLaunchKernelGGL(k_ctl_end, dim3(rb), dim3(64), 0, s, d);
    return hipGetLastError();
}

// Capture `slots` pass slots and the remaining-RVE count in one graph.
hipError_t build_graph(BatchHost *h)
{
    if (h->exec) {
        (void)hipGraphExecDestroy(h->exec);
        h->exec = nullptr;
    }
    if (h->graph) {
        (void)hipGraphDestroy(h->graph);
        h->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int i = 0; i < h->slots && e == hipSuccess; ++i) e = enqueue_slot(h);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, h->stream, h->d.remaining);
        hipLaunchKernelGGL(k_count_remaining, dim3(nblk(h->d.count, 64)), dim3(64), 0, h->stream,
                           h->d);
        e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->stream, &g);
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    h->graph = g;
    return hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
}

}  // namespace

struct srm_batch {
    BatchHost h;
};

extern "C" {

const char *srm_batch_last_error(void) { return g_batch_error.c_str(); }

srm_status srm_batch_init(int32_t count, const srm_params *params, const double *pos,
                          const double *rho, srm_batch **out)
{
    if (count < 1 || !params || !pos || !out) return bfail(SRM_EINVAL, "bad arguments");
    int64_t ntotal = 0, ncells = 0;
    for (int32_t r = 0; r < count; ++r) {
        const srm_params &p = params[r];
        if ((p.dim != 2 && p.dim != 3) || p.shape != SRM_BALL)
            return bfail(SRM_EINVAL, "RVE %d: balls in 2D or 3D only", r);
        if (p.n < 1 || p.n_k < 1 || p.n_k > 32767 || p.n_l < 0 || p.n_l > 255)
            return bfail(SRM_EINVAL, "RVE %d: bad n, n_k or n_l", r);
        if (!(p.s_target >= 0.0) || !(p.c_w >= 0.0) || !(p.c_m >= 0.0))
            return bfail(SRM_EINVAL, "RVE %d: bad scales", r);
        for (int a = 0; a < p.dim; ++a)
            if (!(p.box[a] > 0.0)) return bfail(SRM_EINVAL, "RVE %d: box edge <= 0", r);
        ntotal += p.n;
        ncells += p.n + 2;
    }
    if (ncells > 0x7fffffffLL) return bfail(SRM_EINVAL, "ensemble too large");
    srm_batch *b = new (std::nothrow) srm_batch();
    if (!b) return bfail(SRM_ENOMEM, "host allocation failed");
    BatchHost *h = &b->h;
    auto bail = [&](srm_status st) {
        for (void *v : h->allocs) (void)hipFree(v);
        if (h->hrem) (void)hipHostFree(h->hrem);
        for (hipEvent_t ev : h->done)
            if (ev) (void)hipEventDestroy(ev);
        if (h->stream) (void)hipStreamDestroy(h->stream);
        delete b;
        return st;
    };
    if (hipStreamCreate(&h->stream) != hipSuccess) return bail(bfail(SRM_EDEVICE, "stream"));
    h->poly = rho != nullptr;
    BatchDev &d = h->d;
    d.count = count;
    d.wave_occ = kWaveOccupancy;
    d.ntotal = (int32_t)ntotal;
    d.ncells = (int32_t)ncells;
    hipError_t e = hipSuccess;
    for (int set = 0; set < 3 && !e; ++set) {
        for (int a = 0; a < 3 && !e; ++a) e = balloc(h, &d.x[set][a], (size_t)ntotal);
        if (!e) e = balloc(h, &d.id[set], (size_t)ntotal);
        if (!e && h->poly) e = balloc(h, &d.rho[set], (size_t)ntotal);
    }
    if (!e) e = balloc(h, &d.rve, (size_t)count);
    if (!e) e = balloc(h, &d.rve_of, (size_t)ntotal);
    if (!e) e = balloc(h, &d.rve_of_cell, (size_t)ncells);
    if (!e) e = balloc(h, &d.cell, (size_t)ntotal);
    if (!e) e = balloc(h, &d.slot, (size_t)ntotal);
    if (!e) e = balloc(h, &d.tmpid, (size_t)ntotal);
    if (!e) e = balloc(h, &d.counts, (size_t)ncells);
    if (!e) e = balloc(h, &d.start, (size_t)ncells + 1);
    if (!e) e = balloc(h, &d.partials, (size_t)(ncells / 2048 + 2));
    if (!e) e = balloc(h, &d.acc, (size_t)ntotal);
    if (!e) e = balloc(h, &d.failed, (size_t)ntotal + 1);
    if (!e) e = balloc(h, &d.prefix, (size_t)32 * (count + 1));
    if (!e) e = balloc(h, &d.remaining, 1);
    if (e) return bail(bfail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    if (hipHostMalloc((void **)&h->hrem, sizeof(int32_t) * kDepth, hipHostMallocDefault) !=
        hipSuccess)
        return bail(bfail(SRM_ENOMEM, "pinned allocation failed"));
    for (hipEvent_t &ev : h->done)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return bail(bfail(SRM_EDEVICE, "event"));

    // control records, particle -> RVE maps, initial P in set 0 (id order,
    // binned by the first pass slot of each sweep)
    h->init.resize(count);
    std::vector<int32_t> rve_of((size_t)ntotal), rve_of_cell((size_t)ncells);
    std::vector<int32_t> ids((size_t)ntotal);
    std::vector<double> xs[3];
    for (int a = 0; a < 3; ++a) xs[a].assign((size_t)ntotal, 0.0);
    int64_t off = 0, coff = 0, poff = 0;
    for (int32_t r = 0; r < count; ++r) {
        const srm_params &p = params[r];
        Rve v{};
        v.dim = p.dim;
        v.n = (int32_t)p.n;
        v.off = (int32_t)off;
        v.coff = (int32_t)coff;
        v.n_k = p.n_k;
        v.n_l = p.n_l;
        v.poly = h->poly ? 1 : 0;
        for (int a = 0; a < 3; ++a) v.box[a] = (a < p.dim) ? p.box[a] : 1.0;
        v.s_target = p.s_target;
        v.c_w = p.c_w;
        v.c_m = p.c_m;
        v.key0 = (uint32_t)p.seed;
        v.key1 = (uint32_t)(p.seed >> 32);
        v.ncap = even_cap(p.dim, p.n);
        v.s = 0.0;
        v.t = 0;
        v.mode = kSweepStart;
        v.role[kRoleP] = 0;
        v.role[kRoleQ] = 1;
        v.role[kRoleT] = 2;
        v.rho_max = 1.0;
        if (h->poly) {
            double m = 0.0;
            for (int64_t i = 0; i < p.n; ++i) m = rho[off + i] > m ? rho[off + i] : m;
            v.rho_max = m;
        }
        for (int64_t i = 0; i < p.n; ++i) {
            rve_of[(size_t)(off + i)] = r;
            ids[(size_t)(off + i)] = (int32_t)i;
            for (int a = 0; a < p.dim; ++a) {
                const double x = pos[poff + a * p.n + i];
                if (!(x >= 0.0 && x < p.box[a]))
                    return bail(bfail(SRM_EINVAL, "RVE %d: coordinate outside the box", r));
                xs[a][(size_t)(off + i)] = x;
            }
        }
        for (int64_t c = 0; c < p.n + 2; ++c) rve_of_cell[(size_t)(coff + c)] = r;
        h->init[r] = v;
        // colour-cell bound per dimension class: n/2^dim + 1 per RVE
        h->bound[p.dim == 3 ? 1 : 0] += (int32_t)(p.n / (p.dim == 3 ? 8 : 4) + 1);
        off += p.n;
        coff += p.n + 2;
        poff += (int64_t)p.dim * p.n;
    }
    const size_t nb = (size_t)ntotal;
    if (hipMemcpy(d.rve_of, rve_of.data(), nb * 4, hipMemcpyHostToDevice) ||
        hipMemcpy(d.rve_of_cell, rve_of_cell.data(), (size_t)ncells * 4, hipMemcpyHostToDevice) ||
        hipMemcpy(d.id[0], ids.data(), nb * 4, hipMemcpyHostToDevice) ||
        hipMemcpy(d.x[0][0], xs[0].data(), nb * 8, hipMemcpyHostToDevice) ||
        hipMemcpy(d.x[0][1], xs[1].data(), nb * 8, hipMemcpyHostToDevice) ||
        hipMemcpy(d.x[0][2], xs[2].data(), nb * 8, hipMemcpyHostToDevice) ||
        (h->poly && hipMemcpy(d.rho[0], rho, nb * 8, hipMemcpyHostToDevice)))
        return bail(bfail(SRM_EDEVICE, "upload failed"));
    if (hipMemcpy(d.rve, h->init.data(), sizeof(Rve) * count, hipMemcpyHostToDevice))
        return bail(bfail(SRM_EDEVICE, "upload failed"));
    *out = b;
    return SRM_OK;
}

srm_status srm_batch_configure(srm_batch *b, int32_t slots_per_replay, int32_t block,
                               int32_t wave_occupancy)
{
    if (!b || slots_per_replay < 1 || slots_per_replay > 64 ||
        (block != 64 && block != 128 && block != 256) ||
        wave_occupancy < 1 || wave_occupancy > 64)
        return bfail(SRM_EINVAL, "bad configuration");
    b->h.slots = slots_per_replay;
    b->h.block = block;
    b->h.d.wave_occ = wave_occupancy;
    if (b->h.exec) {
        (void)hipGraphExecDestroy(b->h.exec);
        b->h.exec = nullptr;
    }
    return SRM_OK;
}

srm_status srm_batch_run(srm_batch *b, int32_t max_sweeps, srm_batch_info *info)
{
    if (!b || max_sweeps < 0) return bfail(SRM_EINVAL, "bad arguments");
    BatchHost *h = &b->h;
    // set the sweep budget of every RVE
    std::vector<Rve> cur(h->d.count);
    BHIP(hipMemcpy(cur.data(), h->d.rve, sizeof(Rve) * h->d.count, hipMemcpyDeviceToHost));
    for (auto &v : cur) {
        v.max_sweeps = v.sweeps + max_sweeps;
        if (v.mode == kNotConv) v.mode = kSweepStart;
    }
    BHIP(hipMemcpy(h->d.rve, cur.data(), sizeof(Rve) * h->d.count, hipMemcpyHostToDevice));
    if (!h->exec) BHIP(build_graph(h));
    // Up to kDepth replays are queued ahead, each followed by a copy of its
    // count of unfinished RVEs into its own pinned slot and an event.  The
    // host waits for the oldest replay only, so the device never idles on
    // the host's check; once a count reads 0 nothing more is queued.  A
    // replay after the last RVE finished changes nothing (every RVE is
    // inactive), so the few already queued behind it are harmless.
    int64_t replays = 0, retired = 0;
    bool finished = false;
    while (!finished) {
        while (replays - retired < kDepth) {
            const int slot = (int)(replays % kDepth);
            BHIP(hipGraphLaunch(h->exec, h->stream));
            BHIP(hipMemcpyAsync(h->hrem + slot, h->d.remaining, sizeof(int32_t),
                                hipMemcpyDeviceToHost, h->stream));
            BHIP(hipEventRecord(h->done[slot], h->stream));
            ++replays;
        }
        const int slot = (int)(retired % kDepth);
        BHIP(hipEventSynchronize(h->done[slot]));
        finished = h->hrem[slot] == 0;
        ++retired;
    }
    BHIP(hipStreamSynchronize(h->stream));
    BHIP(hipMemcpy(cur.data(), h->d.rve, sizeof(Rve) * h->d.count, hipMemcpyDeviceToHost));
    int32_t done = 0, notconv = 0;
    int64_t passes = 0, updates = 0;
    for (auto &v : cur) {
        done += (v.mode == kDone || (v.mode == kSweepStart && !(v.s < v.s_target)));
        notconv += v.mode == kNotConv;
        passes += v.passes;
        updates += (int64_t)v.passes * v.n;
    }
    if (info) {
        info->replays = replays;
        info->slots = replays * h->slots;
        info->converged = done;
        info->not_converged = notconv;
        info->passes = passes;
        info->updates = updates;
    }
    return notconv ? bfail(SRM_ENOTCONV, "%d RVEs did not converge", notconv) : SRM_OK;
}

srm_status srm_batch_get(srm_batch *b, int32_t r, double *pos, double *s, int64_t *sweep,
                         int64_t *passes)
{
    if (!b || r < 0 || r >= b->h.d.count) return bfail(SRM_EINVAL, "bad arguments");
    BatchHost *h = &b->h;
    Rve v;
    BHIP(hipMemcpy(&v, h->d.rve + r, sizeof(Rve), hipMemcpyDeviceToHost));
    if (pos) {
        const int set = v.role[kRoleP];
        std::vector<int32_t> id((size_t)v.n);
        std::vector<double> x((size_t)v.n);
        BHIP(hipMemcpy(id.data(), h->d.id[set] + v.off, (size_t)v.n * 4, hipMemcpyDeviceToHost));
        for (int a = 0; a < v.dim; ++a) {
            BHIP(hipMemcpy(x.data(), h->d.x[set][a] + v.off, (size_t)v.n * 8,
                           hipMemcpyDeviceToHost));
            for (int32_t i = 0; i < v.n; ++i) pos[(size_t)a * v.n + id[i]] = x[i];
        }
    }
    if (s) *s = v.s;
    if (sweep) *sweep = v.t;
    if (passes) *passes = v.passes;
    return SRM_OK;
}

srm_status srm_batch_free(srm_batch *b)
{
    if (!b) return SRM_OK;
    BatchHost *h = &b->h;
    (void)hipStreamSynchronize(h->stream);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (void *v : h->allocs) (void)hipFree(v);
    if (h->hrem) (void)hipHostFree(h->hrem);
    for (hipEvent_t ev : h->done)
        if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(h->stream);
    delete b;
    return SRM_OK;
}

}  // extern "C"
