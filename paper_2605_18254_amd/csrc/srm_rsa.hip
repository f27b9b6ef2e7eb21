// srm_rsa.hip -- random sequential addition (RSA) on the GPU: the
// non-overlapping start at a low volume fraction f0 that Sec. 2 and
// Algorithm 1 take as the input of the swelling loop.
//
// Classical RSA is sequential: candidate k (a Philox-drawn point, plus a
// unit normal for platelets) is kept when it meets none of the particles
// kept before it, and gets the next id.  The GPU reproduces that sequence
// exactly, a batch of M candidates at a time:
//   1. draw the batch and test every candidate against the particles kept
//      in earlier batches (cell grid, 3^d stencil); survivors keep k order;
//   2. bin the survivors and decide them by rounds: a survivor is kept once
//      every earlier survivor that it meets is rejected, and rejected once
//      one of them is kept (the earliest undecided survivor always decides,
//      so every round makes progress);
//   3. number the kept survivors in k order after the particles placed so
//      far (dropping those beyond n) and re-bin the kept set.
// Which candidates are kept depends only on k order, never on M.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

#include "srm_internal.hpp"

namespace srm {
namespace {

constexpr int kRsaBlock = 256;

unsigned rsa_blocks(int64_t n) { return (unsigned)((n + kRsaBlock - 1) / kRsaBlock); }

// 53-bit uniform in [0, 1) from the top 27 bits of wa and the top 26 of wb
// (every operation exact).
__device__ __forceinline__ double u53(uint32_t wa, uint32_t wb)
{
    return ((double)(wa >> 5) * 67108864.0 + (double)(wb >> 6)) * 0x1p-53;
}

// Candidate k: centre from Philox counters (k_lo, k_hi, call, 2) -- axes 0, 1
// from call 0, axis 2 from call 1 -- scaled by the box, a product that rounds
// up to L folded to 0; platelets add Algorithm 3's random direction of length
// 1 on stream 3 (counter (k_lo, k_hi, attempt, 3)).
template <int DIM, bool PLATE>
__device__ __forceinline__ void rsa_candidate(uint32_t key0, uint32_t key1, uint64_t k,
                                              const Grid &g, double x[3], double nrm[3])
{
    const uint32_t klo = (uint32_t)k, khi = (uint32_t)(k >> 32);
    uint32_t w0 = klo, w1 = khi, w2 = 0u, w3 = 2u;
    philox4x32_10(w0, w1, w2, w3, key0, key1);
    x[0] = u53(w0, w1) * g.box[0];
    x[1] = u53(w2, w3) * g.box[1];
    x[2] = 0.0;
    if (DIM == 3) {
        uint32_t v0 = klo, v1 = khi, v2 = 1u, v3 = 2u;
        philox4x32_10(v0, v1, v2, v3, key0, key1);
        x[2] = u53(v0, v1) * g.box[2];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        if (x[a] >= g.box[a]) x[a] = 0.0;
    if (PLATE) {
        const Draw d{key0, key1, khi, 0u};
        unit_vector<3>(d, klo, 3u, 1.0, nrm);
    }
}

// Do particle (y, ny) -- the earlier one -- and (x, nx) meet?  Balls: the
// squared minimum-image distance of x - y against (R + R)^2; platelets: the
// disk test with the earlier particle as disk 1.
template <int DIM, bool PLATE>
__device__ __forceinline__ bool rsa_meet(const Grid &g, const double x[3], const double nx[3],
                                         double y0, double y1, double y2, const double ny[3],
                                         double radius, double sig2)
{
    const double d0 = min_image(x[0] - y0, g.box[0], g.half[0]);
    const double d1 = min_image(x[1] - y1, g.box[1], g.half[1]);
    if (PLATE) {
        const double d2 = min_image(x[2] - y2, g.box[2], g.half[2]);
        return disks_intersect(d0, d1, d2, ny, radius, nx, radius);
    }
    double q = d0 * d0 + d1 * d1;
    if (DIM == 3) {
        const double d2 = min_image(x[2] - y2, g.box[2], g.half[2]);
        q = q + d2 * d2;
    }
    return q <= sig2;
}

template <int DIM>
__device__ __forceinline__ void cell_coords(const Grid &g, const double x[3], int32_t &cx,
                                            int32_t &cy, int32_t &cz)
{
    cx = cell_coord(x[0], g.inv_w[0], g.na[0]);
    cy = cell_coord(x[1], g.inv_w[1], g.na[1]);
    cz = (DIM == 3) ? cell_coord(x[2], g.inv_w[2], g.na[2]) : 0;
}

// Step 1: draw candidates k0 .. k0+m-1, test each against the kept set
// (cell-sorted `kept`, ranges `start`), store it and its survival flag.
template <int DIM, bool PLATE>
__global__ void __launch_bounds__(kRsaBlock)
    k_rsa_draw(uint32_t key0, uint32_t key1, uint64_t k0, int32_t m, Grid g, PBuf kept,
               const int32_t *__restrict__ start, int32_t nkept, double radius, double sig2,
               PBuf cand, int32_t *__restrict__ alive)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double x[3], nx[3] = {0.0, 0.0, 0.0};
    rsa_candidate<DIM, PLATE>(key0, key1, k0 + (uint64_t)j, g, x, nx);
    bool hit = false;
    if (nkept > 0) {
        int32_t cx, cy, cz;
        cell_coords<DIM>(g, x, cx, cy, cz);
        int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
        stencil_slices<DIM>(g, start, cx, cy, cz, lo, hi);
        for (int r = 0; r < Rows<DIM>::kRanges && !hit; ++r) {
            for (int32_t q = lo[r]; q < hi[r]; ++q) {
                double ny[3] = {0.0, 0.0, 0.0};
                if (PLATE) {
                    ny[0] = kept.nrm[0][q];
                    ny[1] = kept.nrm[1][q];
                    ny[2] = kept.nrm[2][q];
                }
                if (rsa_meet<DIM, PLATE>(g, x, nx, kept.x[0][q], kept.x[1][q],
                                         DIM == 3 ? kept.x[2][q] : 0.0, ny, radius, sig2)) {
                    hit = true;
                    break;
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) cand.x[a][j] = x[a];
    if (PLATE) {
        cand.nrm[0][j] = nx[0];
        cand.nrm[1][j] = nx[1];
        cand.nrm[2][j] = nx[2];
    }
    alive[j] = hit ? 0 : 1;
}

// Survivors in k order: record s = off[j] takes candidate j.
__global__ void __launch_bounds__(kRsaBlock)
    k_rsa_compact(int32_t m, int dim, const int32_t *__restrict__ alive,
                  const int32_t *__restrict__ off, PBuf cand, PBuf surv,
                  int32_t *__restrict__ surv_j, int32_t *__restrict__ state)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || !alive[j]) return;
    const int32_t s = off[j];
    for (int a = 0; a < dim; ++a) surv.x[a][s] = cand.x[a][j];
    if (cand.nrm[0]) {
        surv.nrm[0][s] = cand.nrm[0][j];
        surv.nrm[1][s] = cand.nrm[1][j];
        surv.nrm[2][s] = cand.nrm[2][j];
    }
    surv.id[s] = s;
    surv_j[s] = j;
    state[s] = 0;
}

// Step 2, one round over the cell-sorted survivors `ss`: an undecided
// survivor is rejected (2) if an earlier survivor that it meets is kept (1),
// kept if every such survivor is rejected, else it waits; waiting survivors
// are counted in *pending.  States only move from 0 to a final value, so a
// state read while another lane writes it is either still 0 (wait) or final.
template <int DIM, bool PLATE>
__global__ void __launch_bounds__(kRsaBlock)
    k_rsa_round(int32_t ns, Grid g, PBuf ss, const int32_t *__restrict__ start, double radius,
                double sig2, int32_t *state, int32_t *__restrict__ pending)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ns) return;
    const int32_t me = ss.id[p];
    if (__hip_atomic_load(&state[me], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    double x[3] = {ss.x[0][p], ss.x[1][p], DIM == 3 ? ss.x[2][p] : 0.0};
    double nx[3] = {0.0, 0.0, 0.0};
    if (PLATE) {
        nx[0] = ss.nrm[0][p];
        nx[1] = ss.nrm[1][p];
        nx[2] = ss.nrm[2][p];
    }
    int32_t cx, cy, cz;
    cell_coords<DIM>(g, x, cx, cy, cz);
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(g, start, cx, cy, cz, lo, hi);
    bool wait = false, out = false;
    for (int r = 0; r < Rows<DIM>::kRanges && !out; ++r) {
        for (int32_t q = lo[r]; q < hi[r]; ++q) {
            const int32_t other = ss.id[q];
            if (other >= me) continue;
            double ny[3] = {0.0, 0.0, 0.0};
            if (PLATE) {
                ny[0] = ss.nrm[0][q];
                ny[1] = ss.nrm[1][q];
                ny[2] = ss.nrm[2][q];
            }
            if (!rsa_meet<DIM, PLATE>(g, x, nx, ss.x[0][q], ss.x[1][q],
                                      DIM == 3 ? ss.x[2][q] : 0.0, ny, radius, sig2))
                continue;
            const int32_t st =
                __hip_atomic_load(&state[other], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (st == 1) {
                out = true;
                break;
            }
            if (st == 0) wait = true;
        }
    }
    if (out) __hip_atomic_store(&state[me], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (!wait) __hip_atomic_store(&state[me], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else atomicAdd(pending, 1);
}

__global__ void __launch_bounds__(kRsaBlock)
    k_rsa_keepflag(int32_t ns, const int32_t *__restrict__ state, int32_t *__restrict__ flag)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) flag[s] = state[s] == 1 ? 1 : 0;
}

// Step 3: kept survivor s with rank r < room becomes particle placed + r;
// its record goes to the caller's id-order arrays and the id-order kept set.
// The last one placed records its candidate index + 1 in *drawn.
__global__ void __launch_bounds__(kRsaBlock)
    k_rsa_place(int32_t ns, int dim, const int32_t *__restrict__ state,
                const int32_t *__restrict__ rank, int32_t room, int32_t placed, uint64_t k0,
                PBuf surv, const int32_t *__restrict__ surv_j, PBuf out, int64_t *__restrict__ src,
                unsigned long long *__restrict__ drawn)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns || state[s] != 1) return;
    const int32_t r = rank[s];
    if (r >= room) return;
    const int32_t id = placed + r;
    for (int a = 0; a < dim; ++a) out.x[a][id] = surv.x[a][s];
    if (surv.nrm[0]) {
        out.nrm[0][id] = surv.nrm[0][s];
        out.nrm[1][id] = surv.nrm[1][s];
        out.nrm[2][id] = surv.nrm[2][s];
    }
    out.id[id] = id;
    const uint64_t k = k0 + (uint64_t)surv_j[s];
    if (src) src[id] = (int64_t)k;
    if (r == room - 1) *drawn = (unsigned long long)(k + 1);
}

thread_local std::string g_rsa_error;

srm_status rfail(srm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
srm_status rfail(srm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_rsa_error = buf;
    set_last_error(buf);
    return st;
}

#define RHIP(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return rfail(SRM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// Device buffers of one RSA call, freed on every exit.
struct RsaArena {
    std::vector<void *> p;
    ~RsaArena()
    {
        for (void *q : p) (void)hipFree(q);
    }
    template <class T_>
    hipError_t get(T_ **ptr, size_t count)
    {
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, (count > 0 ? count : 1) * sizeof(T_));
        if (e == hipSuccess) {
            p.push_back(v);
            *ptr = (T_ *)v;
        }
        return e;
    }
};

template <int DIM, bool PLATE>
hipError_t launch_draw(uint32_t k0key, uint32_t k1key, uint64_t k0, int32_t m, const Grid &g,
                       const PBuf &kept, const int32_t *start, int32_t nkept, double radius,
                       double sig2, const PBuf &cand, int32_t *alive, hipStream_t st)
{
    hipLaunchKernelGGL((k_rsa_draw<DIM, PLATE>), dim3(rsa_blocks(m)), dim3(kRsaBlock), 0, st,
                       k0key, k1key, k0, m, g, kept, start, nkept, radius, sig2, cand, alive);
    return hipGetLastError();
}

template <int DIM, bool PLATE>
hipError_t launch_round(int32_t ns, const Grid &g, const PBuf &ss, const int32_t *start,
                        double radius, double sig2, int32_t *state, int32_t *pending,
                        hipStream_t st)
{
    hipLaunchKernelGGL((k_rsa_round<DIM, PLATE>), dim3(rsa_blocks(ns)), dim3(kRsaBlock), 0, st,
                       ns, g, ss, start, radius, sig2, state, pending);
    return hipGetLastError();
}

}  // namespace
}  // namespace srm

using namespace srm;

extern "C" srm_status srm_rsa(int32_t dim, int32_t shape, int64_t n, const double *box,
                              double radius, uint64_t seed, int64_t max_candidates,
                              int64_t batch, double *pos, double *normals, int64_t *src,
                              int32_t mem_kind, void *hip_stream, srm_rsa_info *info)
{
    if (dim != 2 && dim != 3) return rfail(SRM_EINVAL, "dim must be 2 or 3");
    if (shape != SRM_BALL && shape != SRM_PLATELET) return rfail(SRM_EINVAL, "bad shape");
    if (shape == SRM_PLATELET && dim != 3) return rfail(SRM_EINVAL, "platelets are 3D");
    if (n < 0 || n > 0x7fffffffLL) return rfail(SRM_EINVAL, "n out of range");
    if (!box) return rfail(SRM_EINVAL, "box is NULL");
    for (int a = 0; a < dim; ++a)
        if (!(box[a] > 0.0) || !isfinite(box[a])) return rfail(SRM_EINVAL, "box edge <= 0");
    if (!(radius >= 0.0) || !isfinite(radius)) return rfail(SRM_EINVAL, "bad radius");
    if (max_candidates < 0) return rfail(SRM_EINVAL, "max_candidates < 0");
    if (batch < 0 || batch > (1LL << 28)) return rfail(SRM_EINVAL, "batch out of range");
    if (mem_kind != SRM_MEM_HOST && mem_kind != SRM_MEM_DEVICE)
        return rfail(SRM_EINVAL, "bad mem_kind");
    if (n > 0 && !pos) return rfail(SRM_EINVAL, "pos is NULL");
    if (n > 0 && shape == SRM_PLATELET && !normals)
        return rfail(SRM_EINVAL, "platelets need a normals buffer");
    const bool plate = shape == SRM_PLATELET;
    hipStream_t st = (hipStream_t)hip_stream;
    srm_rsa_info inf{};
    if (n == 0) {
        if (info) *info = inf;
        return SRM_OK;
    }
    const int32_t nn = (int32_t)n;

    double box3[3] = {box[0], box[1], dim == 3 ? box[2] : 1.0};
    // Cells at least 2.5 radii wide: two particles that meet have centres
    // within 2 radii, so they sit in neighbouring cells.
    const Grid g = sweep_grid(dim, box3, even_cap(dim, n), 0.0, radius);
    const int64_t mmax = batch > 0 ? batch : std::max<int64_t>(65536, std::min<int64_t>(2 * n, 1LL << 25));

    RsaArena ar;
    PBuf out{}, kept{}, cand{}, surv{}, ss{};
    int32_t *alive = nullptr, *off = nullptr, *surv_j = nullptr, *state = nullptr,
            *flag = nullptr, *rank = nullptr, *pending = nullptr;
    unsigned long long *drawn_d = nullptr;
    Counters *cnt = nullptr;
    Scratch sc{};
    const int64_t pmax = std::max<int64_t>(n, mmax);
    sc.cap = g.ncell;
    hipError_t e = hipSuccess;
    auto take = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    for (int a = 0; a < dim; ++a) {
        if (mem_kind == SRM_MEM_DEVICE) out.x[a] = pos + (size_t)a * (size_t)n;
        else take(ar.get(&out.x[a], (size_t)n));
        take(ar.get(&kept.x[a], (size_t)n));
        take(ar.get(&cand.x[a], (size_t)mmax));
        take(ar.get(&surv.x[a], (size_t)mmax));
        take(ar.get(&ss.x[a], (size_t)mmax));
    }
    if (plate) {
        for (int a = 0; a < 3; ++a) {
            if (mem_kind == SRM_MEM_DEVICE) out.nrm[a] = normals + (size_t)a * (size_t)n;
            else take(ar.get(&out.nrm[a], (size_t)n));
            take(ar.get(&kept.nrm[a], (size_t)n));
            take(ar.get(&cand.nrm[a], (size_t)mmax));
            take(ar.get(&surv.nrm[a], (size_t)mmax));
            take(ar.get(&ss.nrm[a], (size_t)mmax));
        }
    }
    int64_t *src_d = nullptr;
    if (src) {
        if (mem_kind == SRM_MEM_DEVICE) src_d = src;
        else take(ar.get(&src_d, (size_t)n));
    }
    take(ar.get(&out.id, (size_t)n));
    take(ar.get(&kept.id, (size_t)n));
    take(ar.get(&surv.id, (size_t)mmax));
    take(ar.get(&ss.id, (size_t)mmax));
    take(ar.get(&alive, (size_t)mmax));
    take(ar.get(&off, (size_t)mmax + 1));
    take(ar.get(&surv_j, (size_t)mmax));
    take(ar.get(&state, (size_t)mmax));
    take(ar.get(&flag, (size_t)mmax));
    take(ar.get(&rank, (size_t)mmax + 1));
    take(ar.get(&pending, 1));
    take(ar.get(&drawn_d, 1));
    take(ar.get(&cnt, 1));
    take(ar.get(&sc.cell, (size_t)pmax));
    take(ar.get(&sc.slot, (size_t)pmax));
    take(ar.get(&sc.tmpid, (size_t)pmax));
    take(ar.get(&sc.counts, (size_t)g.ncell + 1));
    take(ar.get(&sc.start, (size_t)g.ncell + 1));
    take(ar.get(&sc.partials, (size_t)(std::max<int64_t>(pmax, g.ncell) / 2048 + 2)));
    if (e != hipSuccess)
        return rfail(SRM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    RHIP(launch_zero_counters(cnt, st));
    RHIP(launch_fill_i32(sc.start, (int64_t)g.ncell + 1, 0, st));

    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const double sig = radius + radius, sig2 = sig * sig;
    int64_t k0 = 0;
    int32_t placed = 0;
    double acc_rate = 1.0;
    int64_t drawn = 0;
    while (placed < nn) {
        if (k0 >= max_candidates) {
            drawn = max_candidates;
            break;
        }
        int64_t m = mmax;
        if (batch == 0) {
            const double want = 1.15 * (double)(nn - placed) / acc_rate + 1024.0;
            m = std::min<int64_t>(mmax, (int64_t)want);
        }
        m = std::min<int64_t>(m, max_candidates - k0);
        const int32_t mi = (int32_t)m;
        // 1. draw and test against the kept set (sc.start holds its ranges)
        if (dim == 3) {
            if (plate)
                RHIP((launch_draw<3, true>(key0, key1, (uint64_t)k0, mi, g, kept, sc.start, placed,
                                           radius, sig2, cand, alive, st)));
            else
                RHIP((launch_draw<3, false>(key0, key1, (uint64_t)k0, mi, g, kept, sc.start,
                                            placed, radius, sig2, cand, alive, st)));
        } else {
            RHIP((launch_draw<2, false>(key0, key1, (uint64_t)k0, mi, g, kept, sc.start, placed,
                                        radius, sig2, cand, alive, st)));
        }
        RHIP(scan_counts(alive, off, sc.partials, mi, st));
        hipLaunchKernelGGL(k_rsa_compact, dim3(rsa_blocks(mi)), dim3(kRsaBlock), 0, st, mi, dim,
                           alive, off, cand, surv, surv_j, state);
        RHIP(hipGetLastError());
        int32_t ns = 0;
        RHIP(hipMemcpyAsync(&ns, off + mi, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RHIP(hipStreamSynchronize(st));
        inf.batches++;
        int32_t kept_now = 0;
        if (ns > 0) {
            // 2. rounds over the binned survivors
            RHIP(bin_particles(dim, surv, ss, ns, g, sc, cnt, st));
            for (int32_t round = 0;; ++round) {
                if (round > ns) return rfail(SRM_EDEVICE, "RSA ordering rounds did not settle");
                RHIP(launch_fill_i32(pending, 1, 0, st));
                if (dim == 3) {
                    if (plate)
                        RHIP((launch_round<3, true>(ns, g, ss, sc.start, radius, sig2, state,
                                                    pending, st)));
                    else
                        RHIP((launch_round<3, false>(ns, g, ss, sc.start, radius, sig2, state,
                                                     pending, st)));
                } else {
                    RHIP((launch_round<2, false>(ns, g, ss, sc.start, radius, sig2, state, pending,
                                                 st)));
                }
                int32_t left = 0;
                RHIP(hipMemcpyAsync(&left, pending, sizeof(int32_t), hipMemcpyDeviceToHost, st));
                RHIP(hipStreamSynchronize(st));
                inf.rounds++;
                if (left == 0) break;
            }
            // 3. number the kept survivors and place them
            hipLaunchKernelGGL(k_rsa_keepflag, dim3(rsa_blocks(ns)), dim3(kRsaBlock), 0, st, ns,
                               state, flag);
            RHIP(hipGetLastError());
            RHIP(scan_counts(flag, rank, sc.partials, ns, st));
            RHIP(hipMemcpyAsync(&kept_now, rank + ns, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            RHIP(hipStreamSynchronize(st));
            const int32_t room = std::min<int32_t>(kept_now, nn - placed);
            if (room > 0) {
                hipLaunchKernelGGL(k_rsa_place, dim3(rsa_blocks(ns)), dim3(kRsaBlock), 0, st, ns,
                                   dim, state, rank, room, placed, (uint64_t)k0, surv, surv_j,
                                   out, src_d, drawn_d);
                RHIP(hipGetLastError());
            }
            placed += room;
        }
        acc_rate = std::max(0.02, (double)kept_now / (double)mi);
        k0 += m;
        if (placed == nn) {
            unsigned long long dd = 0;
            RHIP(hipMemcpyAsync(&dd, drawn_d, sizeof(dd), hipMemcpyDeviceToHost, st));
            RHIP(hipStreamSynchronize(st));
            drawn = (int64_t)dd;
            break;
        }
        // re-bin the kept set for the next batch
        RHIP(bin_particles(dim, out, kept, placed, g, sc, cnt, st));
    }
    if (mem_kind == SRM_MEM_HOST && placed > 0) {
        for (int a = 0; a < dim; ++a)
            RHIP(hipMemcpyAsync(pos + (size_t)a * (size_t)n, out.x[a], (size_t)placed * sizeof(double),
                                hipMemcpyDeviceToHost, st));
        if (plate)
            for (int a = 0; a < 3; ++a)
                RHIP(hipMemcpyAsync(normals + (size_t)a * (size_t)n, out.nrm[a],
                                    (size_t)placed * sizeof(double), hipMemcpyDeviceToHost, st));
        if (src)
            RHIP(hipMemcpyAsync(src, src_d, (size_t)placed * sizeof(int64_t), hipMemcpyDeviceToHost,
                                st));
    }
    RHIP(hipStreamSynchronize(st));
    inf.drawn = drawn;
    inf.placed = placed;
    if (info) *info = inf;
    if (placed < nn)
        return rfail(SRM_ENOTCONV, "%d of %lld particles placed after %lld candidates", placed,
                     (long long)n, (long long)drawn);
    return SRM_OK;
}
