// k_bin.hip -- Algorithm 2 (build cell list) as a counting sort on gfx950:
// cell ids + per-cell counts, an exclusive prefix scan of the counts
// (wavefront shuffles, LDS for the wave totals), then placement into
// cell-sorted SoA arrays with ascending particle ids inside each cell (the
// atomic slot order is not deterministic; the order within a cell is part
// of the sequential processing order): the ids are scattered in arrival
// order, and each particle's rank among its cell's ids gives its slot.
#include "srm_internal.hpp"

namespace srm {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // elements per scan block

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

__global__ void k_fill_u8(uint8_t *a, int64_t n, uint8_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

__global__ void k_zero_counters(Counters *c)
{
    if (threadIdx.x == 0) {
        c->overlap = 0;
        c->bad = 0;
        c->unused = 0;
    }
}

// Trials a pass ran: the accepted trial's index, or N_l for a rejection.
__global__ void __launch_bounds__(kBlock) k_count_trials(const uint8_t *__restrict__ acc, int32_t n,
                                                         int32_t n_l,
                                                         unsigned long long *total)
{
    unsigned long long sum = 0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t c = acc[i];
        sum += (unsigned long long)(c ? c : n_l);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((threadIdx.x & 63) == 0 && sum)
        atomicAdd(total, sum);
}

// Sum of n non-negative counts in 64 bits (*total must start at 0).
__global__ void __launch_bounds__(kBlock) k_sum_i32(const int32_t *__restrict__ a, int32_t n,
                                                    unsigned long long *total)
{
    unsigned long long sum = 0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        sum += (unsigned long long)(uint32_t)a[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((threadIdx.x & 63) == 0 && sum)
        atomicAdd(total, sum);
}

__global__ void k_iota(int32_t *a, int32_t n)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

// Cell id of each particle, its rank in the cell, and a range check of the
// coordinates (a coordinate outside [0, L) or NaN sets cnt->bad and is
// binned into cell 0 so that every index stays in bounds).  The input is in
// the previous cell order, so neighbouring lanes mostly share a cell: each
// run of equal cells within a wavefront claims its slots with one atomic
// add by its first lane.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_bin_count(const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, int32_t n,
                                                      Grid g, int32_t *__restrict__ cell,
                                                      int32_t *__restrict__ slot,
                                                      int32_t *__restrict__ counts, Counters *cnt)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < n;
    int32_t c = -1;
    if (live) {
        const double px = x[p], py = y[p], pz = (DIM == 3) ? z[p] : 0.0;
        bool ok = (px >= 0.0 && px < g.box[0]) && (py >= 0.0 && py < g.box[1]);
        if (DIM == 3) ok = ok && (pz >= 0.0 && pz < g.box[2]);
        c = 0;
        if (ok) c = cell_of<DIM>(g, px, py, pz);
        else cnt->bad = 1;
    }
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(c, 1, 64);
    const bool head = live && (lane == 0 || prev != c);
    const unsigned long long heads = __ballot(head);
    const int nlive = __popcll(__ballot(live));  // live lanes are a prefix
    // first lane of this lane's run, and the run's end
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const unsigned long long below = heads & upto;
    const int first = below ? 63 - __clzll(below) : lane;
    const unsigned long long above = heads & ~upto;
    int next = above ? __ffsll((long long)above) - 1 : 64;
    if (next > nlive) next = nlive;
    int32_t base = 0;
    if (head) base = atomicAdd(&counts[c], next - lane);
    base = __shfl(base, first, 64);
    if (!live) return;
    cell[p] = c;
    slot[p] = base + (lane - first);
}

// Inclusive scan over the 64 lanes of a wavefront.
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ int32_t wave_sum(int32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive scan of one value per thread over a block of kBlock threads;
// returns the prefix of the calling thread and sets *total.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *lds_waves,
                                                        int32_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int kWaves = kBlock / 64;
    const int32_t inc = wave_inclusive_scan(v);
    if (lane == 63) lds_waves[wid] = inc;
    __syncthreads();
    int32_t wave_off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int32_t s = lds_waves[w];
        if (w < wid) wave_off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wave_off + inc - v;
}

// A thread's kScanItems consecutive counts, as two 16-byte loads when the
// array is 16-byte aligned and the run lies wholly inside it.
__device__ __forceinline__ void load_items(const int32_t *__restrict__ in, int64_t base, int32_t m,
                                           bool vec, int32_t v[kScanItems])
{
    static_assert(kScanItems == 8, "two int4 per thread");
    if (vec && base + kScanItems <= m) {
        const int4 a = *reinterpret_cast<const int4 *>(in + base);
        const int4 b = *reinterpret_cast<const int4 *>(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < m) ? in[base + k] : 0;
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_partials(const int32_t *__restrict__ in,
                                                          int32_t m, int32_t *__restrict__ partials)
{
    __shared__ int32_t lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const bool vec = ((uintptr_t)in & 15) == 0;
    int32_t v[kScanItems];
    load_items(in, base, m, vec, v);
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
        partials[blockIdx.x] = t;
    }
}

// Single block: exclusive scan of the per-block sums in place, total into
// out_total.
__global__ void __launch_bounds__(kBlock) k_scan_top(int32_t *__restrict__ partials, int32_t nb,
                                                     int32_t *__restrict__ out_total)
{
    __shared__ int32_t lds[kBlock / 64];
    int32_t carry = 0;
    for (int32_t base = 0; base < nb; base += kBlock) {
        const int32_t i = base + threadIdx.x;
        const int32_t v = (i < nb) ? partials[i] : 0;
        int32_t tot;
        const int32_t ex = block_exclusive_scan(v, lds, &tot);
        if (i < nb) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *out_total = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_final(const int32_t *__restrict__ in, int32_t m,
                                                       const int32_t *__restrict__ partials,
                                                       int32_t *__restrict__ out)
{
    __shared__ int32_t lds[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const bool vec = ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 15) == 0;
    int32_t v[kScanItems];
    load_items(in, base, m, vec, v);
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    int32_t tot;
    int32_t run = partials[blockIdx.x] + block_exclusive_scan(s, lds, &tot);
    int32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (vec && base + kScanItems <= m) {
        *reinterpret_cast<int4 *>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<int4 *>(out + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < m) out[base + k] = o[k];
    }
}

// Placement without a sort pass: the ids go to their cells in arrival order,
// then each particle counts the smaller ids of its cell (its place in
// ascending id order) and moves its record there.
__global__ void __launch_bounds__(kBlock) k_scatter_id(const int32_t *__restrict__ id, int32_t n,
                                                       const int32_t *__restrict__ cell,
                                                       const int32_t *__restrict__ slot,
                                                       const int32_t *__restrict__ start,
                                                       int32_t *__restrict__ tmpid)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    tmpid[start[cell[p]] + slot[p]] = id[p];
}

__global__ void __launch_bounds__(kBlock) k_rank_scatter(PBuf src, PBuf dst, int32_t n, int dim,
                                                         const int32_t *__restrict__ cell,
                                                         const int32_t *__restrict__ start,
                                                         const int32_t *__restrict__ tmpid)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t c = cell[p];
    const int32_t b = start[c], e = start[c + 1];
    const int32_t me = src.id[p];
    int32_t rank = 0;
    for (int32_t q = b; q < e; ++q) rank += tmpid[q] < me;
    const int32_t d = b + rank;
    dst.x[0][d] = src.x[0][p];
    dst.x[1][d] = src.x[1][p];
    if (dim == 3) dst.x[2][d] = src.x[2][p];
    dst.id[d] = me;
    if (src.rho) dst.rho[d] = src.rho[p];
    if (src.nrm[0]) {
        dst.nrm[0][d] = src.nrm[0][p];
        dst.nrm[1][d] = src.nrm[1][p];
        dst.nrm[2][d] = src.nrm[2][p];
    }
}

struct XPtrs {
    const double *x[6];
};

__global__ void __launch_bounds__(kBlock) k_to_id_order(XPtrs xs, int nx, const int32_t *__restrict__ id,
                                                        int32_t n, double *__restrict__ out)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = id[p];
    for (int a = 0; a < nx; ++a) out[(int64_t)a * n + i] = xs.x[a][p];
}

__global__ void __launch_bounds__(kBlock) k_u8_to_id_order(const uint8_t *__restrict__ a,
                                                           const int32_t *__restrict__ id, int32_t n,
                                                           uint8_t *__restrict__ out)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    out[id[p]] = a[p];
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cells_by_id(PBuf b, int32_t n, Grid g, int32_t *__restrict__ out)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    out[b.id[p]] = cell_of<DIM>(g, b.x[0][p], b.x[1][p], DIM == 3 ? b.x[2][p] : 0.0);
}

inline unsigned blocks_for(int64_t n, int per = kBlock)
{
    int64_t b = (n + per - 1) / per;
    return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

hipError_t launch_fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    unsigned nb = blocks_for(n);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3(nb), dim3(kBlock), 0, stream, a, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *a, int64_t n, uint8_t v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    unsigned nb = blocks_for(n);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill_u8, dim3(nb), dim3(kBlock), 0, stream, a, n, v);
    return hipGetLastError();
}

hipError_t count_trials(const uint8_t *acc, int32_t n, int32_t n_l,
                        unsigned long long *total, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int32_t blocks = (n + kBlock - 1) / kBlock < 1024 ? (n + kBlock - 1) / kBlock : 1024;
    hipLaunchKernelGGL(k_count_trials, dim3(blocks), dim3(kBlock), 0, stream, acc, n, n_l, total);
    return hipGetLastError();
}

hipError_t sum_counts64(const int32_t *a, int32_t n, unsigned long long *total,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, (int32_t *)total, (int64_t)2, 0);
    if (n <= 0) return hipGetLastError();
    const int32_t blocks = (n + kBlock - 1) / kBlock < 1024 ? (n + kBlock - 1) / kBlock : 1024;
    hipLaunchKernelGGL(k_sum_i32, dim3(blocks), dim3(kBlock), 0, stream, a, n, total);
    return hipGetLastError();
}

hipError_t launch_zero_counters(Counters *c, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, c);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *a, int32_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(n)), dim3(kBlock), 0, stream, a, n);
    return hipGetLastError();
}

hipError_t scan_counts(const int32_t *counts, int32_t *start, int32_t *partials, int32_t m,
                       hipStream_t stream)
{
    const unsigned nb = blocks_for(m, kScanTile);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kBlock), 0, stream, counts, m, partials);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, stream, partials, (int32_t)nb,
                       start + m);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kBlock), 0, stream, counts, m, partials,
                       start);
    return hipGetLastError();
}

hipError_t bin_particles(int dim, const PBuf &src, const PBuf &dst, int32_t n, const Grid &g,
                         Scratch &sc, Counters *cnt, hipStream_t stream)
{
    if ((int64_t)g.ncell > sc.cap) return hipErrorInvalidValue;
    hipError_t e = launch_fill_i32(sc.counts, g.ncell, 0, stream);
    if (e != hipSuccess) return e;
    if (n > 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_bin_count<3>, dim3(blocks_for(n)), dim3(kBlock), 0, stream,
                               src.x[0], src.x[1], src.x[2], n, g, sc.cell, sc.slot, sc.counts,
                               cnt);
        else
            hipLaunchKernelGGL(k_bin_count<2>, dim3(blocks_for(n)), dim3(kBlock), 0, stream,
                               src.x[0], src.x[1], src.x[2], n, g, sc.cell, sc.slot, sc.counts,
                               cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = scan_counts(sc.counts, sc.start, sc.partials, g.ncell, stream)) != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter_id, dim3(blocks_for(n)), dim3(kBlock), 0, stream, src.id, n,
                           sc.cell, sc.slot, sc.start, sc.tmpid);
        hipLaunchKernelGGL(k_rank_scatter, dim3(blocks_for(n)), dim3(kBlock), 0, stream, src, dst,
                           n, dim, sc.cell, sc.start, sc.tmpid);
    }
    return hipGetLastError();
}

hipError_t to_id_order(const double *const *x, int nx, const int32_t *id, int32_t n, double *out,
                       hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    XPtrs xs{};
    for (int a = 0; a < nx && a < 6; ++a) xs.x[a] = x[a];
    hipLaunchKernelGGL(k_to_id_order, dim3(blocks_for(n)), dim3(kBlock), 0, stream, xs, nx, id, n,
                       out);
    return hipGetLastError();
}

hipError_t u8_to_id_order(const uint8_t *a, const int32_t *id, int32_t n, uint8_t *out,
                          hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_u8_to_id_order, dim3(blocks_for(n)), dim3(kBlock), 0, stream, a, id, n,
                       out);
    return hipGetLastError();
}

hipError_t cells_by_id(int dim, const PBuf &b, int32_t n, const Grid &g, int32_t *out,
                       hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    if (dim == 3)
        hipLaunchKernelGGL(k_cells_by_id<3>, dim3(blocks_for(n)), dim3(kBlock), 0, stream, b, n, g,
                           out);
    else
        hipLaunchKernelGGL(k_cells_by_id<2>, dim3(blocks_for(n)), dim3(kBlock), 0, stream, b, n, g,
                           out);
    return hipGetLastError();
}

}  // namespace srm
