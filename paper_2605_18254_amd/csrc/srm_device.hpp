// srm_device.hpp -- device-side building blocks of the SRM sweep on gfx950:
// counter-based random numbers, the random unit vector of Algorithm 3,
// periodic wrap (Algorithm 4), minimum image (Algorithm 5), cell coordinates
// (Algorithm 2) and the thin-disk intersection predicate (Sec. 3.3).
//
// Every expression is written so that, compiled with -ffp-contract=off,
// it performs exactly the IEEE binary64 operations of the method's
// definition in the same order (no fused multiply-add), so results agree bit
// for bit with any other correctly rounded evaluation of the same sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srm {

constexpr int kMaxDim = 3;

// Adaptive cell grid of one sweep (cells per axis, reciprocal width, box).
struct Grid {
    int32_t na[3];
    int32_t ncell;
    double inv_w[3];
    double box[3];
    double half[3];  // 0.5 * box[a], exact
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// 4-word multiply/xor bijection with a Weyl-sequence key schedule.  The key
// schedule is the same for every lane, so it stays in scalar registers.
// Each round's two 32x32 -> 64-bit products are written as 64-bit
// multiplies of zero-extended words, which gfx950 issues as one
// v_mad_u64_u32 each instead of a v_mul_lo_u32 / v_mul_hi_u32 pair.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                              uint32_t &x3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        const uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x0 = y0;
        x1 = (uint32_t)p1;
        x2 = y2;
        x3 = (uint32_t)p0;
        k0 += W0;
        k1 += W1;
    }
}

// Odd multiple of 2^-32 in (-1, 1) from a 32-bit word (all steps exact).
__device__ __forceinline__ double sym_uniform(uint32_t w)
{
    return ((double)w - 2147483647.5) * 0x1p-31;
}

// Counter-based draw parameters of one particle's trial moves.
struct Draw {
    uint32_t key0, key1;  // seed
    uint32_t t;           // sweep counter
    uint32_t word;        // kind<<31 | k<<16 | l<<8
};

// Random vector of length `len` with uniform direction.  Each Philox call
// (counter (id, t, word | call, stream)) gives two attempts (v1, v2) in
// (-1,1)^2, kept when s = v1^2 + v2^2 < 1.  3D: Marsaglia's point on the
// sphere (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2s) times len; 2D:
// (v1, v2) * (len / sqrt(s)).
template <int DIM>
__device__ __forceinline__ void unit_vector(const Draw &d, uint32_t id, uint32_t stream,
                                            double len, double v[3])
{
    for (uint32_t r = 0; r < 64; ++r) {
        uint32_t w[4] = {id, d.t, d.word | r, stream};
        philox4x32_10(w[0], w[1], w[2], w[3], d.key0, d.key1);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const double v1 = sym_uniform(w[2 * a]);
            const double v2 = sym_uniform(w[2 * a + 1]);
            const double s = v1 * v1 + v2 * v2;
            if (s < 1.0) {
                if (DIM == 3) {
                    const double h = 2.0 * __builtin_sqrt(1.0 - s);
                    v[0] = (v1 * h) * len;
                    v[1] = (v2 * h) * len;
                    v[2] = (1.0 - 2.0 * s) * len;
                } else {
                    const double g = len / __builtin_sqrt(s);
                    v[0] = v1 * g;
                    v[1] = v2 * g;
                    v[2] = 0.0;
                }
                return;
            }
        }
    }
    v[0] = len;
    v[1] = 0.0;
    v[2] = 0.0;
}

__host__ __device__ __forceinline__ uint32_t counter_word(uint32_t kind, uint32_t k, uint32_t l)
{
    return (kind << 31) | (k << 16) | (l << 8);
}

// Algorithm 4: if x < 0 add L, then if x >= L subtract L.
__device__ __forceinline__ double wrap_coord(double x, double L)
{
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

// Minimum image of Algorithm 5 on one axis (half = 0.5 L).
__device__ __forceinline__ double min_image(double d, double L, double half)
{
    if (d > half) d -= L;
    if (d < -half) d += L;
    return d;
}

// Algorithm 2 cell coordinate: (int)(x * N_a / L_a); the top edge folds to 0.
__device__ __forceinline__ int32_t cell_coord(double x, double inv_w, int32_t na)
{
    int32_t c = (int32_t)(x * inv_w);
    return (c == na) ? 0 : c;
}

template <int DIM>
__device__ __forceinline__ int32_t cell_of(const Grid &g, double x, double y, double z)
{
    const int32_t cx = cell_coord(x, g.inv_w[0], g.na[0]);
    const int32_t cy = cell_coord(y, g.inv_w[1], g.na[1]);
    const int32_t cz = (DIM == 3) ? cell_coord(z, g.inv_w[2], g.na[2]) : 0;
    return cx + g.na[0] * (cy + g.na[1] * cz);
}

// Zero-thickness disk-disk intersection: (c1, n1, a1) is the disk with the
// lower particle id.  d = minimum image of c2 - c1.  Cull on |d| > a1 + a2;
// parallel planes intersect only when coplanar; otherwise both disks must
// reach the planes' common line and their chords on it must overlap.
__device__ __forceinline__ bool disks_intersect(double dx, double dy, double dz,
                                                const double n1[3], double a1,
                                                const double n2[3], double a2)
{
    const double dd = dx * dx + dy * dy + dz * dz;
    const double sa = a1 + a2;
    if (dd > sa * sa) return false;
    const double ux = n1[1] * n2[2] - n1[2] * n2[1];
    const double uy = n1[2] * n2[0] - n1[0] * n2[2];
    const double uz = n1[0] * n2[1] - n1[1] * n2[0];
    const double uu = ux * ux + uy * uy + uz * uz;
    if (uu == 0.0) {
        const double hn = n1[0] * dx + n1[1] * dy + n1[2] * dz;
        return hn == 0.0;
    }
    const double h = n2[0] * dx + n2[1] * dy + n2[2] * dz;
    const double wx = uy * n1[2] - uz * n1[1];
    const double wy = uz * n1[0] - ux * n1[2];
    const double wz = ux * n1[1] - uy * n1[0];
    const double f = h / uu;
    const double px = wx * f, py = wy * f, pz = wz * f;
    const double A = a1 * a1 - (px * px + py * py + pz * pz);
    if (A < 0.0) return false;
    const double ex = dx - px, ey = dy - py, ez = dz - pz;
    const double t0 = (ex * ux + ey * uy + ez * uz) / uu;
    const double B = a2 * a2 - ((ex * ex + ey * ey + ez * ez) - (t0 * t0) * uu);
    if (B < 0.0) return false;
    const double Ap = A / uu, Bp = B / uu, C = t0 * t0;
    const double D = (C - Ap) - Bp;
    if (D <= 0.0) return true;
    return D * D <= (4.0 * Ap) * Bp;
}

// Adaptive grid of Algorithm 1 for the largest radius rmax: cell edge
// cs = 2.5 rmax + 2.5 c_m; per axis N_a = m - (m mod 2) cells if
// m = min(floor(L_a / cs), ncap) >= 4, else one cell.  The same IEEE
// operations on the host and on the device.
__host__ __device__ __forceinline__ Grid sweep_grid(int dim, const double box[3], int64_t ncap,
                                                    double c_m, double rmax)
{
    Grid g{};
    const double cs = 2.5 * rmax + 2.5 * c_m;
    for (int a = 0; a < 3; ++a) {
        g.box[a] = box[a];
        g.half[a] = 0.5 * box[a];
        if (a >= dim) {
            g.na[a] = 1;
            g.inv_w[a] = 1.0 / box[a];
            continue;
        }
        int64_t m;
        const double q = (cs > 0.0) ? box[a] / cs : 0.0;
        if (!(cs > 0.0) || q >= (double)ncap) m = ncap;
        else m = (int64_t)q;
        g.na[a] = (int32_t)((m >= 4) ? m - (m & 1) : 1);
        g.inv_w[a] = (double)g.na[a] / box[a];
    }
    g.ncell = g.na[0] * g.na[1] * g.na[2];
    return g;
}

// Swelling step: s' = min(s + c_w s_target, s_target).
__host__ __device__ __forceinline__ double swell_scale(double s, double c_w, double s_target)
{
    const double s1 = s + c_w * s_target;
    return (s1 < s_target) ? s1 : s_target;
}

// Largest even m with m^dim <= n.
__host__ __device__ __forceinline__ int64_t even_cap(int dim, int64_t n)
{
    int64_t m = 0;
    for (;;) {
        const int64_t c = m + 2;
        int64_t pw = 1;
        for (int a = 0; a < dim; ++a) pw *= c;
        if (pw > n) break;
        m = c;
    }
    return m;
}

// Slices of a cell-sorted array covering the 3^dim cells around a cell.
template <int DIM>
struct Rows {
    static constexpr int kRows = (DIM == 3) ? 9 : 3;
    static constexpr int kRanges = 2 * kRows;  // a row of 3 cells is <= 2 slices
};

__device__ __forceinline__ int32_t wrap_index(int32_t c, int32_t n)
{
    c += (c < 0) ? n : 0;
    c -= (c >= n) ? n : 0;
    return c;
}

// Slices of the cell-sorted arrays covering the 3^dim cells around
// (cx, cy, cz).  Cells (cx-1, cx, cx+1) of one row are consecutive in the
// linear order unless the row wraps, so a row is one slice, or two at the
// x boundary.  Axes with a single cell contribute only offset 0.
template <int DIM>
__device__ __forceinline__ void stencil_slices(const Grid &g, const int32_t *__restrict__ start,
                                               int32_t cx, int32_t cy, int32_t cz, int32_t *lo,
                                               int32_t *hi)
{
    const int32_t na0 = g.na[0], na1 = g.na[1], na2 = g.na[2];
#pragma unroll
    for (int iz = 0; iz < (DIM == 3 ? 3 : 1); ++iz) {
#pragma unroll
        for (int iy = 0; iy < 3; ++iy) {
            const int r = (iz * 3 + iy) * 2;
            lo[r] = hi[r] = lo[r + 1] = hi[r + 1] = 0;
            const int32_t dy = iy - 1, dz = (DIM == 3) ? iz - 1 : 0;
            if (na1 < 4 && dy != 0) continue;
            if (DIM == 3 && na2 < 4 && dz != 0) continue;
            const int32_t yy = wrap_index(cy + dy, na1);
            const int32_t zz = (DIM == 3) ? wrap_index(cz + dz, na2) : 0;
            const int32_t row = na0 * (yy + na1 * zz);
            if (na0 < 4) {
                lo[r] = start[row];
                hi[r] = start[row + 1];
            } else if (cx >= 1 && cx <= na0 - 2) {
                lo[r] = start[row + cx - 1];
                hi[r] = start[row + cx + 2];
            } else if (cx == 0) {
                lo[r] = start[row];
                hi[r] = start[row + 2];
                lo[r + 1] = start[row + na0 - 1];
                hi[r + 1] = start[row + na0];
            } else {
                lo[r] = start[row + na0 - 2];
                hi[r] = start[row + na0];
                lo[r + 1] = start[row];
                hi[r + 1] = start[row + 1];
            }
        }
    }
}

}  // namespace srm
