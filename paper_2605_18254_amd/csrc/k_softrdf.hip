// k_softrdf.hip -- differentiable descriptor of a configuration: the
// Gaussian soft-binned radial distribution g_b and the overlap energy
// E = kappa/2 sum_{i<j} max(0, R_i + R_j - r_ij)^2, with a hand-written
// backward (gradients with respect to every position and radius).
//
// Definitions: bins b < nb of width D = r_c/nb, centres c_b = (b + 1/2) D,
// kernel K_b(r) = exp(-(r - c_b)^2 / (2h^2)) / (h sqrt(2 pi)), h = D, C2
// taper w(r) = 1 - 10t^3 + 15t^4 - 6t^5 with t = (r - r_c)/(4h) on
// [r_c, r_c + 4h]; g_b = norm_b sum_{i<j} K_b(r_ij) w(r_ij) with
// norm_b = V / (N(N-1)/2 * 4 pi c_b^2) (3D; 2D: 2 pi c_b).  The neighbour
// search covers r < r_c + 4h, which must also cover every overlapping pair
// (2 R_max <= r_c + 4h).
//
// Forward: thread (p, row) accumulates the pairs of particle p with the
// larger slots of one stencil row in registers (FP64); blocks reduce bin by
// bin (wavefront shuffles) into partials, and a final kernel sums the
// partials in a fixed order, so the result is the same on every run.
//
// Per pair the 64 Gaussians come from three exponentials: with u_b =
// (r - c_b)/h and c_{b+1} - c_b = h, K_{b+1}/K_b = exp(u_b - 1/2) and
// K_{b-1}/K_b = exp(-u_b - 1/2), and each ratio shrinks by e^-1 per step.
// Starting at the bin nearest r (|u| <= 1/2) both chains only decrease, so
// the products lose about one ulp per step (relative) and reach zero where
// the exponential itself underflows.  Backward: thread (p, row) gathers
// dL/dr_ij * u_ij over the row's neighbours of p -- pairs are recomputed,
// not stored -- and the block adds the rows of each particle in order and
// writes only that particle's gradient (no atomics).
#include "srm_internal.hpp"

namespace srm {
namespace {

constexpr int kBlock = kSoftBlock;
constexpr int kMaxBins = kSoftPartialStride - 1;
constexpr double kInvE = 0.36787944117144233;  // e^-1 rounded to binary64

// The two slices of stencil row `row` (row = iz * 3 + iy: the cells at y
// offset iy - 1 and z offset iz - 1, x offsets -1..1) of cell (cx, cy, cz),
// wrapped like the full stencil; empty when the row's offset is unused on an
// axis with fewer than four cells.
template <int DIM>
__device__ __forceinline__ void stencil_row(const Grid &g, const int32_t *__restrict__ start,
                                            int32_t cx, int32_t cy, int32_t cz, int row,
                                            int32_t lo[2], int32_t hi[2])
{
    const int32_t na0 = g.na[0], na1 = g.na[1], na2 = g.na[2];
    lo[0] = hi[0] = lo[1] = hi[1] = 0;
    const int32_t dy = row % 3 - 1, dz = (DIM == 3) ? row / 3 - 1 : 0;
    if (na1 < 4 && dy != 0) return;
    if (DIM == 3 && na2 < 4 && dz != 0) return;
    const int32_t yy = wrap_index(cy + dy, na1);
    const int32_t zz = (DIM == 3) ? wrap_index(cz + dz, na2) : 0;
    const int32_t base = na0 * (yy + na1 * zz);
    if (na0 < 4) {
        lo[0] = start[base];
        hi[0] = start[base + 1];
    } else if (cx >= 1 && cx <= na0 - 2) {
        lo[0] = start[base + cx - 1];
        hi[0] = start[base + cx + 2];
    } else if (cx == 0) {
        lo[0] = start[base];
        hi[0] = start[base + 2];
        lo[1] = start[base + na0 - 1];
        hi[1] = start[base + na0];
    } else {
        lo[0] = start[base + na0 - 2];
        hi[0] = start[base + na0];
        lo[1] = start[base];
        hi[1] = start[base + 1];
    }
}

struct SoftArgs {
    PBuf buf;              // cell-sorted positions, ids, radii (in rho)
    const int32_t *start;
    Grid g;
    int32_t n;
    int32_t nbins;
    double r_c, h, cut, kappa;
};

__device__ __forceinline__ double taper(double r, double r_c, double h, double *dw)
{
    const double span = 4.0 * h;
    if (r <= r_c) {
        *dw = 0.0;
        return 1.0;
    }
    if (r >= r_c + span) {
        *dw = 0.0;
        return 0.0;
    }
    const double t = (r - r_c) / span;
    const double t2 = t * t, t3 = t2 * t;
    *dw = (-30.0 * t2 + 60.0 * t3 - 30.0 * t2 * t2) / span;
    return 1.0 - 10.0 * t3 + 15.0 * t3 * t - 6.0 * t3 * t2;
}

__host__ __device__ __forceinline__ double soft_norm(int dim, int32_t n, const double box[3],
                                                     double c)
{
    double vol = 1.0;
    for (int a = 0; a < dim; ++a) vol *= box[a];
    const double pairs = 0.5 * (double)n * (double)(n - 1);
    const double shell = (dim == 3) ? 4.0 * M_PI * c * c : 2.0 * M_PI * c;
    return vol / (pairs * shell);
}

template <int DIM>
__device__ __forceinline__ void pair_vector(const SoftArgs &a, int32_t p, int32_t q, double d[3])
{
    d[0] = min_image(a.buf.x[0][p] - a.buf.x[0][q], a.g.box[0], a.g.half[0]);
    d[1] = min_image(a.buf.x[1][p] - a.buf.x[1][q], a.g.box[1], a.g.half[1]);
    d[2] = (DIM == 3) ? min_image(a.buf.x[2][p] - a.buf.x[2][q], a.g.box[2], a.g.half[2]) : 0.0;
}

// Forward.  Task p * kRows + row is particle p against stencil row `row`;
// every pair is taken once, by its lower slot.  A wavefront takes 64 tasks
// at a time (one per lane) and walks their candidates in step, the loop
// running to the longest task's count; pairs within the search radius go
// to the wavefront's LDS queue as (r, w(r)) in (step, lane) order, and the
// squared overlaps into a per-lane sum.  The queue is drained with the lanes
// taking the bins: lane b adds c0 exp(-u_b^2 / 2) w for every queued pair,
// u_b = (r - c_b) / h -- the definition itself, one exponential per (pair,
// bin), and one accumulator per lane.  Blocks write their bin and energy
// sums to a partial in a fixed order, so the result is the same on every
// run.
constexpr int kQueue = 512;  // queued pairs per wavefront

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_soft_fwd(SoftArgs a, double *__restrict__ partial)
{
    constexpr int kRows = Rows<DIM>::kRows;
    constexpr int kWaves = kBlock / 64;
    static_assert(kMaxBins == 64, "one lane per bin");
    __shared__ double qr[kWaves][kQueue], qw[kWaves][kQueue];
    __shared__ double red[kWaves][kMaxBins + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double D = a.r_c / a.nbins;
    const double c0 = 1.0 / (a.h * __builtin_sqrt(2.0 * M_PI));
    const double cb = (lane + 0.5) * D;  // centre of this lane's bin
    double accb = 0.0, accE = 0.0;
    int32_t qn = 0;  // queue length (the same in every lane)
    auto drain = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < a.nbins) {
            for (int32_t j = 0; j < qn; ++j) {
                const double u = (qr[wv][j] - cb) / a.h;
                accb += c0 * exp(-0.5 * u * u) * qw[wv][j];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        qn = 0;
    };
    const int64_t tasks = (int64_t)a.n * kRows;
    const int64_t wave0 = (int64_t)blockIdx.x * kWaves + wv;
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t t0 = wave0 * 64; t0 < tasks; t0 += waves * 64) {
        const int64_t t = t0 + lane;
        int32_t p = 0, s0 = 0, n0 = 0, s1 = 0, n1 = 0;
        double Rp = 0.0;
        if (t < tasks) {
            p = (int32_t)(t / kRows);
            const int row = (int)(t % kRows);
            const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
            const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
            const int32_t cz =
                (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
            int32_t lo[2], hi[2];
            stencil_row<DIM>(a.g, a.start, cx, cy, cz, row, lo, hi);
            s0 = lo[0] > p + 1 ? lo[0] : p + 1;
            s1 = lo[1] > p + 1 ? lo[1] : p + 1;
            n0 = hi[0] > s0 ? hi[0] - s0 : 0;
            n1 = hi[1] > s1 ? hi[1] - s1 : 0;
            Rp = a.buf.rho[p];
        }
        const int32_t trip = n0 + n1;
        int32_t steps = trip;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int32_t v = __shfl_xor(steps, o, 64);
            steps = v > steps ? v : steps;
        }
        for (int32_t it = 0; it < steps; ++it) {
            bool has = false;
            double r = 0.0, w = 0.0;
            if (it < trip) {
                const int32_t q = (it < n0) ? s0 + it : s1 + (it - n0);
                double d[3];
                pair_vector<DIM>(a, p, q, d);
                r = __builtin_sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                const double ov = Rp + a.buf.rho[q] - r;
                if (ov > 0.0) accE += ov * ov;
                if (r < a.cut) {
                    double dw;
                    w = taper(r, a.r_c, a.h, &dw);
                    has = true;
                }
            }
            const unsigned long long m = __ballot(has);
            if (has) {
                const int32_t idx = qn + __popcll(m & ((1ull << lane) - 1ull));
                qr[wv][idx] = r;
                qw[wv][idx] = w;
            }
            qn += __popcll(m);
            if (qn > kQueue - 64) drain();
        }
    }
    drain();
    // energy: a fixed shuffle tree over the wavefront
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) accE += __shfl_xor(accE, o, 64);
    red[wv][lane] = accb;
    if (lane == 0) red[wv][kMaxBins] = accE;
    __syncthreads();
    if (threadIdx.x <= kMaxBins) {
        double v = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) v += red[w][threadIdx.x];
        partial[(size_t)blockIdx.x * (kMaxBins + 1) + threadIdx.x] = v;
    }
}

// Sum the block partials of one bin per block (bin blockIdx.x; the energy
// is bin kMaxBins): threads take partials k = t, t + 256, ... in order, then
// a fixed tree; g_b = norm_b * sum, E = kappa/2 * sum.
__global__ void __launch_bounds__(256) k_soft_final(const double *__restrict__ partial,
                                                    int32_t nblocks, int32_t nbins, int dim,
                                                    int32_t n, Grid g, double r_c, double kappa,
                                                    double *__restrict__ gout,
                                                    double *__restrict__ energy)
{
    __shared__ double red[256];
    const int b = (blockIdx.x < (unsigned)nbins) ? (int)blockIdx.x : kMaxBins;
    double s = 0.0;
    for (int32_t k = threadIdx.x; k < nblocks; k += 256) s += partial[(size_t)k * (kMaxBins + 1) + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (b == kMaxBins) {
            *energy = 0.5 * kappa * red[0];
        } else {
            const double D = r_c / nbins;
            gout[b] = red[0] * soft_norm(dim, n, g.box, (b + 0.5) * D);
        }
    }
}

// Backward: particle p's gradient gathers dL/dr_pq (q - p)/r over every
// neighbour q, recomputing the pairs (nothing is stored).  Task (p, row)
// again, a wavefront walking 64 tasks in step; the overlap part of a pair
// is added by its task's lane at once, and the pairs within the search
// radius go to the wavefront's queue.  The queue is drained 64 pairs at a
// time with one pair per lane: the bin sum sum_b coef_b K_b (w (-u_b/h) +
// dw) by the ratio chains, up and down from the bin nearest r in one loop
// of nbins - 1 steps (the same length in every lane); then each task's lane
// adds its pairs' f (q - p) in queue order.  Every task's lane writes its
// row sums to LDS and the block adds each particle's rows in row order, so
// the gradient is the same on every run (no atomics).
constexpr int kBwdBlock = 252;  // 28 particles x 9 rows (3D), 84 x 3 (2D)
constexpr int kBwdQueue = 128;

template <int DIM>
__global__ void __launch_bounds__(256) k_soft_bwd(SoftArgs a, const double *__restrict__ dg,
                                                  const double *__restrict__ dE,
                                                  double *__restrict__ gpos,
                                                  double *__restrict__ grad_r)
{
    constexpr int kRows = Rows<DIM>::kRows;
    constexpr int kPer = kBwdBlock / kRows;
    constexpr int kWaves = 4;
    __shared__ double coef[kMaxBins];
    __shared__ double part[4][256];
    __shared__ double qr[kWaves][kBwdQueue], qw[kWaves][kBwdQueue], qdw[kWaves][kBwdQueue];
    __shared__ double qd[kWaves][3][kBwdQueue];
    __shared__ int8_t qown[kWaves][kBwdQueue];
    const double D = a.r_c / a.nbins;
    if (threadIdx.x < a.nbins)
        coef[threadIdx.x] = dg[threadIdx.x] * soft_norm(DIM, a.n, a.g.box, (threadIdx.x + 0.5) * D);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = threadIdx.x % kRows;
    const int32_t p = blockIdx.x * kPer + threadIdx.x / kRows;
    const bool live = p < a.n && threadIdx.x < kPer * kRows;
    const double ge = *dE * a.kappa;
    const double c0 = 1.0 / (a.h * __builtin_sqrt(2.0 * M_PI));
    const double inv_h = 1.0 / a.h;
    double gx = 0.0, gy = 0.0, gz = 0.0, gr = 0.0;
    int32_t qn = 0;
    auto wave_sync = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto drain = [&]() {
        wave_sync();
        for (int32_t c = 0; c < qn; c += 64) {
            const int32_t j = c + lane;
            double f = 0.0;
            if (j < qn) {
                const double r = qr[wv][j], w = qw[wv][j], dw = qdw[wv][j];
                int32_t b0 = (int32_t)(r / a.h);
                b0 = b0 < a.nbins ? b0 : a.nbins - 1;
                const double u0 = (r - (b0 + 0.5) * D) / a.h;
                const double k0 = c0 * exp(-0.5 * u0 * u0);
                double dLdr = coef[b0] * (k0 * (w * (-u0 * inv_h) + dw));
                double ku = k0, ru = exp(u0 - 0.5), uu = u0;
                double kd = k0, rd = exp(-u0 - 0.5), ud = u0;
                for (int32_t k = 1; k < a.nbins; ++k) {
                    if (b0 + k < a.nbins) {
                        ku *= ru;
                        ru *= kInvE;
                        uu -= 1.0;
                        dLdr += coef[b0 + k] * (ku * (w * (-uu * inv_h) + dw));
                    }
                    if (b0 - k >= 0) {
                        kd *= rd;
                        rd *= kInvE;
                        ud += 1.0;
                        dLdr += coef[b0 - k] * (kd * (w * (-ud * inv_h) + dw));
                    }
                }
                f = dLdr / r;
            }
            wave_sync();
            if (j < qn) qr[wv][j] = f;  // reuse: the pair's factor
            wave_sync();
            const int32_t cend = (qn - c < 64) ? qn : c + 64;
            for (int32_t k = c; k < cend; ++k) {
                if (qown[wv][k] == lane) {
                    const double fk = qr[wv][k];
                    gx += fk * qd[wv][0][k];
                    gy += fk * qd[wv][1][k];
                    gz += fk * qd[wv][2][k];
                }
            }
        }
        wave_sync();
        qn = 0;
    };
    int32_t s0 = 0, n0 = 0, s1 = 0, n1 = 0;
    double Rp = 0.0;
    if (live) {
        const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
        const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
        const int32_t cz = (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
        int32_t lo[2], hi[2];
        stencil_row<DIM>(a.g, a.start, cx, cy, cz, row, lo, hi);
        s0 = lo[0];
        n0 = hi[0] - lo[0];
        s1 = lo[1];
        n1 = hi[1] - lo[1];
        Rp = a.buf.rho[p];
    }
    const int32_t trip = n0 + n1;
    int32_t steps = trip;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t v = __shfl_xor(steps, o, 64);
        steps = v > steps ? v : steps;
    }
    for (int32_t it = 0; it < steps; ++it) {
        bool has = false;
        double r = 0.0, w = 0.0, dw = 0.0, d[3] = {0.0, 0.0, 0.0};
        if (it < trip) {
            const int32_t q = (it < n0) ? s0 + it : s1 + (it - n0);
            if (q != p) {
                pair_vector<DIM>(a, p, q, d);
                r = __builtin_sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r != 0.0) {
                    const double ov = Rp + a.buf.rho[q] - r;
                    if (ov > 0.0) {
                        const double fo = (ge * (-ov)) / r;
                        gx += fo * d[0];
                        gy += fo * d[1];
                        gz += fo * d[2];
                        gr += ge * ov;
                    }
                    if (r < a.cut) {
                        w = taper(r, a.r_c, a.h, &dw);
                        has = true;
                    }
                }
            }
        }
        const unsigned long long m = __ballot(has);
        if (has) {
            const int32_t idx = qn + __popcll(m & ((1ull << lane) - 1ull));
            qr[wv][idx] = r;
            qw[wv][idx] = w;
            qdw[wv][idx] = dw;
            qd[wv][0][idx] = d[0];
            qd[wv][1][idx] = d[1];
            qd[wv][2][idx] = d[2];
            qown[wv][idx] = (int8_t)lane;
        }
        qn += __popcll(m);
        if (qn > kBwdQueue - 64) drain();
    }
    drain();
    part[0][threadIdx.x] = gx;
    part[1][threadIdx.x] = gy;
    part[2][threadIdx.x] = gz;
    part[3][threadIdx.x] = gr;
    __syncthreads();
    if (row == 0 && live) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sr = 0.0;
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            sx += part[0][threadIdx.x + k];
            sy += part[1][threadIdx.x + k];
            sz += part[2][threadIdx.x + k];
            sr += part[3][threadIdx.x + k];
        }
        const int32_t id = a.buf.id[p];
        gpos[id] = sx;
        gpos[(size_t)a.n + id] = sy;
        if (DIM == 3) gpos[2 * (size_t)a.n + id] = sz;
        grad_r[id] = sr;
    }
}

}  // namespace

// Forward blocks: one per kBlock particles (each thread then takes about
// kRows tasks); the partial buffers are sized by this count.
int32_t soft_blocks(int32_t n) { return (n + kBlock - 1) / kBlock; }
int32_t soft_partial_stride() { return kMaxBins + 1; }

hipError_t soft_forward(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                        int32_t nbins, double r_c, double kappa, double *partial, double *gout,
                        double *energy, hipStream_t stream)
{
    const double h = r_c / nbins;
    SoftArgs a{b, start, g, n, nbins, r_c, h, r_c + 4.0 * h, kappa};
    const int32_t nb = soft_blocks(n);
    if (nb > 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_soft_fwd<3>, dim3(nb), dim3(kBlock), 0, stream, a, partial);
        else
            hipLaunchKernelGGL(k_soft_fwd<2>, dim3(nb), dim3(kBlock), 0, stream, a, partial);
    }
    hipLaunchKernelGGL(k_soft_final, dim3(nbins + 1), dim3(256), 0, stream, partial, nb, nbins,
                       dim, n, g, r_c, kappa, gout, energy);
    return hipGetLastError();
}

hipError_t soft_backward(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                         int32_t nbins, double r_c, double kappa, const double *dg,
                         const double *dE, double *gpos, double *grad_r, hipStream_t stream)
{
    const double h = r_c / nbins;
    SoftArgs a{b, start, g, n, nbins, r_c, h, r_c + 4.0 * h, kappa};
    if (n <= 0) return hipSuccess;
    const int per = kBwdBlock / ((dim == 3) ? Rows<3>::kRows : Rows<2>::kRows);
    const unsigned nb = (unsigned)((n + per - 1) / per);
    if (dim == 3)
        hipLaunchKernelGGL(k_soft_bwd<3>, dim3(nb), dim3(256), 0, stream, a, dg, dE, gpos, grad_r);
    else
        hipLaunchKernelGGL(k_soft_bwd<2>, dim3(nb), dim3(256), 0, stream, a, dg, dE, gpos, grad_r);
    return hipGetLastError();
}

}  // namespace srm
