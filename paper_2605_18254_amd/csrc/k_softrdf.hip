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
// Forward: one thread per particle accumulates its pairs with larger ids in
// registers (FP64); blocks reduce in a fixed tree order and a final kernel
// sums the block partials in block order, so the result is the same on
// every run.
//
// Per pair the 64 Gaussians come from three exponentials: with u_b =
// (r - c_b)/h and c_{b+1} - c_b = h, K_{b+1}/K_b = exp(u_b - 1/2) and
// K_{b-1}/K_b = exp(-u_b - 1/2), and each ratio shrinks by e^-1 per step.
// Starting at the bin nearest r (|u| <= 1/2) both chains only decrease, so
// the products lose about one ulp per step (relative) and reach zero where
// the exponential itself underflows.  Backward: one thread per particle gathers dL/dr_ij * u_ij over
// all its neighbours -- pairs are recomputed, not stored -- and writes only
// its own gradient (no atomics).
#include "srm_internal.hpp"

namespace srm {
namespace {

constexpr int kBlock = kSoftBlock;
constexpr int kMaxBins = kSoftPartialStride - 1;
constexpr double kInvE = 0.36787944117144233;  // e^-1 rounded to binary64

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

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_soft_fwd(SoftArgs a, double *__restrict__ partial)
{
    __shared__ double red[kBlock];
    double acc[kMaxBins + 1];
#pragma unroll
    for (int b = 0; b <= kMaxBins; ++b) acc[b] = 0.0;
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.n) {
        const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
        const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
        const int32_t cz = (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
        int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
        stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
        const int32_t idp = a.buf.id[p];
        const double Rp = a.buf.rho[p];
        const double c0 = 1.0 / (a.h * __builtin_sqrt(2.0 * M_PI));
        const double D = a.r_c / a.nbins;
        for (int r_ = 0; r_ < Rows<DIM>::kRanges; ++r_) {
            for (int32_t q = lo[r_]; q < hi[r_]; ++q) {
                if (a.buf.id[q] <= idp) continue;
                double d[3];
                pair_vector<DIM>(a, p, q, d);
                const double r = __builtin_sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                const double ov = Rp + a.buf.rho[q] - r;
                if (ov > 0.0) acc[kMaxBins] += ov * ov;
                if (r >= a.cut) continue;
                double dw;
                const double w = taper(r, a.r_c, a.h, &dw);
                int32_t b0 = (int32_t)(r / a.h);
                b0 = b0 < a.nbins ? b0 : a.nbins - 1;
                const double u0 = (r - (b0 + 0.5) * D) / a.h;
                const double k0 = c0 * exp(-0.5 * u0 * u0) * w;
                double ku = k0, ru = exp(u0 - 0.5);
#pragma unroll
                for (int b = 0; b < kMaxBins; ++b) {
                    if (b < a.nbins && b >= b0) {
                        if (b > b0) {
                            ku *= ru;
                            ru *= kInvE;
                        }
                        acc[b] += ku;
                    }
                }
                double kd = k0, rd = exp(-u0 - 0.5);
#pragma unroll
                for (int b = kMaxBins - 1; b >= 0; --b) {
                    if (b < b0) {
                        kd *= rd;
                        rd *= kInvE;
                        acc[b] += kd;
                    }
                }
            }
        }
    }
    // fixed-order tree reduction of every bin over the block
#pragma unroll
    for (int b = 0; b <= kMaxBins; ++b) {
        if (b < a.nbins || b == kMaxBins) {
            red[threadIdx.x] = acc[b];
            __syncthreads();
            for (int s = kBlock / 2; s > 0; s >>= 1) {
                if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) partial[(size_t)blockIdx.x * (kMaxBins + 1) + b] = red[0];
            __syncthreads();
        }
    }
}

// Sum the block partials in block order; g_b = norm_b * sum, E = kappa/2 * sum.
__global__ void k_soft_final(const double *__restrict__ partial, int32_t nblocks, int32_t nbins,
                             int dim, int32_t n, Grid g, double r_c, double kappa,
                             double *__restrict__ gout, double *__restrict__ energy)
{
    const int b = threadIdx.x;
    if (b > kMaxBins) return;
    if (b < nbins || b == kMaxBins) {
        double s = 0.0;
        for (int32_t k = 0; k < nblocks; ++k) s += partial[(size_t)k * (kMaxBins + 1) + b];
        if (b == kMaxBins) {
            *energy = 0.5 * kappa * s;
        } else {
            const double D = r_c / nbins;
            gout[b] = s * soft_norm(dim, n, g.box, (b + 0.5) * D);
        }
    }
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_soft_bwd(SoftArgs a, const double *__restrict__ dg,
                                                     const double *__restrict__ dE,
                                                     double *__restrict__ gpos,
                                                     double *__restrict__ grad_r)
{
    __shared__ double coef[kMaxBins];
    const double D = a.r_c / a.nbins;
    if (threadIdx.x < a.nbins)
        coef[threadIdx.x] = dg[threadIdx.x] * soft_norm(DIM, a.n, a.g.box, (threadIdx.x + 0.5) * D);
    __syncthreads();
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const double ge = *dE * a.kappa;
    const int32_t cx = cell_coord(a.buf.x[0][p], a.g.inv_w[0], a.g.na[0]);
    const int32_t cy = cell_coord(a.buf.x[1][p], a.g.inv_w[1], a.g.na[1]);
    const int32_t cz = (DIM == 3) ? cell_coord(a.buf.x[2][p], a.g.inv_w[2], a.g.na[2]) : 0;
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
    const double Rp = a.buf.rho[p];
    const double c0 = 1.0 / (a.h * __builtin_sqrt(2.0 * M_PI));
    double gx = 0.0, gy = 0.0, gz = 0.0, gr = 0.0;
    for (int r_ = 0; r_ < Rows<DIM>::kRanges; ++r_) {
        for (int32_t q = lo[r_]; q < hi[r_]; ++q) {
            if (q == p) continue;
            double d[3];
            pair_vector<DIM>(a, p, q, d);
            const double r = __builtin_sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r == 0.0) continue;
            double dLdr = 0.0;
            const double ov = Rp + a.buf.rho[q] - r;
            if (ov > 0.0) {
                dLdr += ge * (-ov);
                gr += ge * ov;
            }
            if (r < a.cut) {
                double dw;
                const double w = taper(r, a.r_c, a.h, &dw);
                // d/dr [K_b w] = K_b (w (-u_b / h) + dw), K_b by the chains above
                int32_t b0 = (int32_t)(r / a.h);
                b0 = b0 < a.nbins ? b0 : a.nbins - 1;
                const double u0 = (r - (b0 + 0.5) * D) / a.h;
                const double k0 = c0 * exp(-0.5 * u0 * u0);
                const double inv_h = 1.0 / a.h;
                dLdr += coef[b0] * (k0 * (w * (-u0 * inv_h) + dw));
                double ku = k0, ru = exp(u0 - 0.5), uu = u0;
                for (int32_t b = b0 + 1; b < a.nbins; ++b) {
                    ku *= ru;
                    ru *= kInvE;
                    uu -= 1.0;
                    dLdr += coef[b] * (ku * (w * (-uu * inv_h) + dw));
                }
                double kd = k0, rd = exp(-u0 - 0.5), ud = u0;
                for (int32_t b = b0 - 1; b >= 0; --b) {
                    kd *= rd;
                    rd *= kInvE;
                    ud += 1.0;
                    dLdr += coef[b] * (kd * (w * (-ud * inv_h) + dw));
                }
            }
            const double f = dLdr / r;
            gx += f * d[0];
            gy += f * d[1];
            gz += f * d[2];
        }
    }
    const int32_t id = a.buf.id[p];
    gpos[id] = gx;
    gpos[(size_t)a.n + id] = gy;
    if (DIM == 3) gpos[2 * (size_t)a.n + id] = gz;
    grad_r[id] = gr;
}

}  // namespace

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
    hipLaunchKernelGGL(k_soft_final, dim3(1), dim3(kMaxBins + 1), 0, stream, partial, nb, nbins,
                       dim, n, g, r_c, kappa, gout, energy);
    return hipGetLastError();
}

hipError_t soft_backward(int dim, const PBuf &b, const int32_t *start, const Grid &g, int32_t n,
                         int32_t nbins, double r_c, double kappa, const double *dg,
                         const double *dE, double *gpos, double *grad_r, hipStream_t stream)
{
    const double h = r_c / nbins;
    SoftArgs a{b, start, g, n, nbins, r_c, h, r_c + 4.0 * h, kappa};
    const int32_t nb = soft_blocks(n);
    if (nb <= 0) return hipSuccess;
    if (dim == 3)
        hipLaunchKernelGGL(k_soft_bwd<3>, dim3(nb), dim3(kBlock), 0, stream, a, dg, dE, gpos,
                           grad_r);
    else
        hipLaunchKernelGGL(k_soft_bwd<2>, dim3(nb), dim3(kBlock), 0, stream, a, dg, dE, gpos,
                           grad_r);
    return hipGetLastError();
}

}  // namespace srm
