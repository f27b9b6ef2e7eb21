// k_pairs.hip -- neighbour enumeration of a committed configuration: the
// contact / gap pairs (srm_pairs) and the histogram of centre distances
// (srm_rdf).  Both bin the particles into their own grid whose cells are at
// least as wide as the cutoff, so every pair within the cutoff lies in the
// 3^dim stencil; a pair (i, j) is evaluated once, by the thread of the lower
// id i, as the minimum image of x_i - x_j.
#include "srm_internal.hpp"

namespace srm {
namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b > 0 ? b : 1);
}

struct PairArgs {
    PBuf buf;          // cell-sorted particles
    const int32_t *start;
    Grid g;
    int32_t n;
    int32_t shape;
    double tau;        // spherodisks: half-thickness / outer radius (0: zero-thickness disks)
    double s;          // radius scale
    double gap;
};

// The pair predicate for the particle in slot p (the lower id) and slot q.
template <int DIM>
__device__ __forceinline__ bool pair_hit(const PairArgs &a, int32_t p, int32_t q)
{
    const double Rp = a.buf.rho ? a.s * a.buf.rho[p] : a.s;
    const double Rq = a.buf.rho ? a.s * a.buf.rho[q] : a.s;
    if (a.shape == SRM_PLATELET) {
        // disk 1 = lower id (p): d = minimum image of c2 - c1
        const double ex = min_image(a.buf.x[0][q] - a.buf.x[0][p], a.g.box[0], a.g.half[0]);
        const double ey = min_image(a.buf.x[1][q] - a.buf.x[1][p], a.g.box[1], a.g.half[1]);
        const double ez = min_image(a.buf.x[2][q] - a.buf.x[2][p], a.g.box[2], a.g.half[2]);
        const double n1[3] = {a.buf.nrm[0][p], a.buf.nrm[1][p], a.buf.nrm[2][p]};
        const double n2[3] = {a.buf.nrm[0][q], a.buf.nrm[1][q], a.buf.nrm[2][q]};
        // zero thickness: radii grown by gap / 2 in their planes; spherodisks:
        // shells grown by gap / 2 around each surface
        if (a.tau == 0.0)
            return disks_intersect(ex, ey, ez, n1, Rp + 0.5 * a.gap, n2, Rq + 0.5 * a.gap);
        return spherodisks_overlap(ex, ey, ez, n1, Rp, n2, Rq, a.tau, a.gap);
    }
    const double dx = min_image(a.buf.x[0][p] - a.buf.x[0][q], a.g.box[0], a.g.half[0]);
    const double dy = min_image(a.buf.x[1][p] - a.buf.x[1][q], a.g.box[1], a.g.half[1]);
    double qq = dx * dx + dy * dy;
    if (DIM == 3) {
        const double dz = min_image(a.buf.x[2][p] - a.buf.x[2][q], a.g.box[2], a.g.half[2]);
        qq = qq + dz * dz;
    }
    const double sig = (Rp + Rq) + a.gap;
    return qq <= sig * sig;
}

// EMIT = false: rowcnt[id_p] = number of partners with a larger id.
// EMIT = true: their ids into partner[rowoff[id_p] ...] (unsorted).
template <int DIM, bool EMIT>
__global__ void __launch_bounds__(kBlock) k_pairs(PairArgs a, int32_t *__restrict__ rowcnt,
                                                  const int32_t *__restrict__ rowoff,
                                                  int32_t *__restrict__ partner)
{
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
    const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
    const int32_t cz = (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
    const int32_t idp = a.buf.id[p];
    int32_t k = 0, base = EMIT ? rowoff[idp] : 0;
#pragma unroll
    for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
        for (int32_t q = lo[r]; q < hi[r]; ++q) {
            const int32_t idq = a.buf.id[q];
            if (idq <= idp) continue;
            if (pair_hit<DIM>(a, p, q)) {
                if (EMIT) partner[base + k] = idq;
                ++k;
            }
        }
    }
    if (!EMIT) rowcnt[idp] = k;
}

// Row i of the pair list: sort its partner ids and write (i, j) pairs.
__global__ void __launch_bounds__(kBlock) k_pairs_rows(int32_t n, const int32_t *__restrict__ rowoff,
                                                       int32_t *__restrict__ partner,
                                                       int32_t *__restrict__ ij)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = rowoff[i], e = rowoff[i + 1];
    for (int32_t u = b + 1; u < e; ++u) {
        const int32_t key = partner[u];
        int32_t v = u - 1;
        while (v >= b && partner[v] > key) {
            partner[v + 1] = partner[v];
            --v;
        }
        partner[v + 1] = key;
    }
    for (int32_t u = b; u < e; ++u) {
        ij[2 * (int64_t)u] = i;
        ij[2 * (int64_t)u + 1] = partner[u];
    }
}

// Distance histogram: bin b = (int)(sqrt(q) * inv) for pairs with id_p <
// id_q and b < nbins.  Per-block counts in LDS when nbins fits, else direct
// 64-bit atomics; integer counts are order-independent.
template <int DIM, bool SHARED>
__global__ void __launch_bounds__(kBlock) k_rdf(PairArgs a, int32_t nbins, double inv,
                                                unsigned long long *__restrict__ counts)
{
    extern __shared__ uint32_t hist[];
    if (SHARED) {
        for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0;
        __syncthreads();
    }
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.n) {
        const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
        const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
        const int32_t cz = (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
        int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
        stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
        const int32_t idp = a.buf.id[p];
        const double xp = a.buf.x[0][p], yp = a.buf.x[1][p];
        const double zp = (DIM == 3) ? a.buf.x[2][p] : 0.0;
#pragma unroll
        for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
            for (int32_t q = lo[r]; q < hi[r]; ++q) {
                if (a.buf.id[q] <= idp) continue;
                const double dx = min_image(xp - a.buf.x[0][q], a.g.box[0], a.g.half[0]);
                const double dy = min_image(yp - a.buf.x[1][q], a.g.box[1], a.g.half[1]);
                double qq = dx * dx + dy * dy;
                if (DIM == 3) {
                    const double dz = min_image(zp - a.buf.x[2][q], a.g.box[2], a.g.half[2]);
                    qq = qq + dz * dz;
                }
                const double x = __builtin_sqrt(qq) * inv;
                if (x < (double)nbins) {
                    const int32_t b = (int32_t)x;
                    if (b < nbins) {
                        if (SHARED) atomicAdd(&hist[b], 1u);
                        else atomicAdd(&counts[b], 1ull);
                    }
                }
            }
        }
    }
    if (SHARED) {
        __syncthreads();
        for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x)
            if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
    }
}

// Nearest neighbour of the particle in slot p within r2 = r_max^2: the
// minimum of q over the stencil (order-independent), written by id; then
// its histogram bin (LDS counts when nbins fits, else direct atomics).
template <int DIM, bool SHARED>
__global__ void __launch_bounds__(kBlock) k_nearest(PairArgs a, double r2, double *__restrict__ dist,
                                                    int32_t nbins, double inv,
                                                    unsigned long long *__restrict__ counts)
{
    extern __shared__ uint32_t hist[];
    if (SHARED) {
        for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0;
        __syncthreads();
    }
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.n) {
        const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
        const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
        const int32_t cz = (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
        int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
        stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
        const double xp = a.buf.x[0][p], yp = a.buf.x[1][p];
        const double zp = (DIM == 3) ? a.buf.x[2][p] : 0.0;
        double best = r2;
        bool found = false;
#pragma unroll
        for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
            for (int32_t q = lo[r]; q < hi[r]; ++q) {
                if (q == p) continue;
                const double dx = min_image(xp - a.buf.x[0][q], a.g.box[0], a.g.half[0]);
                const double dy = min_image(yp - a.buf.x[1][q], a.g.box[1], a.g.half[1]);
                double qq = dx * dx + dy * dy;
                if (DIM == 3) {
                    const double dz = min_image(zp - a.buf.x[2][q], a.g.box[2], a.g.half[2]);
                    qq = qq + dz * dz;
                }
                if (qq < best) {
                    best = qq;
                    found = true;
                }
            }
        }
        const double d = found ? __builtin_sqrt(best) : __builtin_inf();
        if (dist) dist[a.buf.id[p]] = d;
        if (counts && found) {
            const double x = d * inv;
            if (x < (double)nbins) {
                const int32_t b = (int32_t)x;
                if (b < nbins) {
                    if (SHARED) atomicAdd(&hist[b], 1u);
                    else atomicAdd(&counts[b], 1ull);
                }
            }
        }
    }
    if (SHARED) {
        __syncthreads();
        for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x)
            if (hist[b]) atomicAdd(&counts[b], (unsigned long long)hist[b]);
    }
}

}  // namespace

hipError_t pairs_count(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                       int shape, double tau, double s, double gap, int32_t *rowcnt,
                       hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const PairArgs a{b, start, g, n, shape, tau, s, gap};
    if (dim == 3)
        hipLaunchKernelGGL((k_pairs<3, false>), dim3(blocks_for(n)), dim3(kBlock), 0, stream, a,
                           rowcnt, nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_pairs<2, false>), dim3(blocks_for(n)), dim3(kBlock), 0, stream, a,
                           rowcnt, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t pairs_emit(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                      int shape, double tau, double s, double gap, const int32_t *rowoff,
                      int32_t *partner, int32_t *ij, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const PairArgs a{b, start, g, n, shape, tau, s, gap};
    if (dim == 3)
        hipLaunchKernelGGL((k_pairs<3, true>), dim3(blocks_for(n)), dim3(kBlock), 0, stream, a,
                           nullptr, rowoff, partner);
    else
        hipLaunchKernelGGL((k_pairs<2, true>), dim3(blocks_for(n)), dim3(kBlock), 0, stream, a,
                           nullptr, rowoff, partner);
    hipLaunchKernelGGL(k_pairs_rows, dim3(blocks_for(n)), dim3(kBlock), 0, stream, n, rowoff,
                       partner, ij);
    return hipGetLastError();
}

hipError_t rdf_counts(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                      int32_t nbins, double inv, unsigned long long *counts, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const PairArgs a{b, start, g, n, SRM_BALL, 0.0, 0.0};
    const bool shared = nbins <= 8192;
    const size_t lds = shared ? (size_t)nbins * sizeof(uint32_t) : 0;
    if (dim == 3) {
        if (shared) hipLaunchKernelGGL((k_rdf<3, true>), dim3(blocks_for(n)), dim3(kBlock), lds,
                                       stream, a, nbins, inv, counts);
        else hipLaunchKernelGGL((k_rdf<3, false>), dim3(blocks_for(n)), dim3(kBlock), 0, stream,
                                a, nbins, inv, counts);
    } else {
        if (shared) hipLaunchKernelGGL((k_rdf<2, true>), dim3(blocks_for(n)), dim3(kBlock), lds,
                                       stream, a, nbins, inv, counts);
        else hipLaunchKernelGGL((k_rdf<2, false>), dim3(blocks_for(n)), dim3(kBlock), 0, stream,
                                a, nbins, inv, counts);
    }
    return hipGetLastError();
}

hipError_t nearest(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                   double r_max, double *dist, int32_t nbins, unsigned long long *counts,
                   hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const PairArgs a{b, start, g, n, SRM_BALL, 0.0, 0.0};
    const double r2 = r_max * r_max;
    const double inv = counts ? (double)nbins / r_max : 0.0;
    const bool shared = counts && nbins <= 8192;
    const size_t lds = shared ? (size_t)nbins * sizeof(uint32_t) : 0;
    if (dim == 3) {
        if (shared) hipLaunchKernelGGL((k_nearest<3, true>), dim3(blocks_for(n)), dim3(kBlock), lds,
                                       stream, a, r2, dist, nbins, inv, counts);
        else hipLaunchKernelGGL((k_nearest<3, false>), dim3(blocks_for(n)), dim3(kBlock), 0,
                                stream, a, r2, dist, nbins, inv, counts);
    } else {
        if (shared) hipLaunchKernelGGL((k_nearest<2, true>), dim3(blocks_for(n)), dim3(kBlock), lds,
                                       stream, a, r2, dist, nbins, inv, counts);
        else hipLaunchKernelGGL((k_nearest<2, false>), dim3(blocks_for(n)), dim3(kBlock), 0,
                                stream, a, r2, dist, nbins, inv, counts);
    }
    return hipGetLastError();
}

}  // namespace srm
