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

// ---- spherodisks (Sec. 3.3's platelet model) ----------------------------
// A spherodisk of outer radius a and thickness t = 2h is the set of points
// within h of a flat core disk of radius A = a - h.  Two overlap iff the
// distance between their core disks is at most h1 + h2 (touching counts).
// Core disk 1: centre 0, unit normal n1, radius A1; core disk 2: centre d.
// The decision uses two certificates:
//  - points p on disk 1 and q on disk 2 with |q - p| <= T prove overlap;
//  - a unit direction u with L(u) = u.d - A1 |u x n1| - A2 |u x n2| > T
//    proves separation (A |u x n| is a disk's half-extent along u), and
//    L((q* - p*)/|q* - p*|) is the distance at the closest pair.
// Candidate pairs come from the zero-thickness test, the point of each rim
// nearest the other plane, alternating projections between the disks and
// Newton's method on the two rim angles; a pair within 1e-12 (A1 + A2) of
// T, or left undecided, counts as overlapping.  Every expression matches
// the oracle's, operation for operation.
__device__ __forceinline__ double sd_lower(const double u[3], const double d[3],
                                           const double n1[3], double A1, const double n2[3],
                                           double A2)
{
    const double x0 = u[1] * n1[2] - u[2] * n1[1];
    const double x1 = u[2] * n1[0] - u[0] * n1[2];
    const double x2 = u[0] * n1[1] - u[1] * n1[0];
    const double y0 = u[1] * n2[2] - u[2] * n2[1];
    const double y1 = u[2] * n2[0] - u[0] * n2[2];
    const double y2 = u[0] * n2[1] - u[1] * n2[0];
    const double e1 = __builtin_sqrt(x0 * x0 + x1 * x1 + x2 * x2);
    const double e2 = __builtin_sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    const double ud = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    return (ud - A1 * e1) - A2 * e2;
}

// Nearest point y of the disk (centre 0, unit normal n, radius A) to x;
// true when it lies on the rim.
__device__ __forceinline__ bool sd_proj(const double x[3], const double n[3], double A,
                                        double y[3])
{
    const double h = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    y[0] = x[0] - h * n[0];
    y[1] = x[1] - h * n[1];
    y[2] = x[2] - h * n[2];
    const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    if (r2 <= A * A) return false;
    const double f = A / __builtin_sqrt(r2);
    y[0] = y[0] * f;
    y[1] = y[1] * f;
    y[2] = y[2] * f;
    return true;
}

// 1: overlap, 0: separated, -1: undecided by the pair (p, q).
__device__ __forceinline__ int sd_certify(const double p[3], const double q[3], const double d[3],
                                          const double n1[3], double A1, const double n2[3],
                                          double A2, double T)
{
    const double w0 = q[0] - p[0], w1 = q[1] - p[1], w2 = q[2] - p[2];
    const double ww = w0 * w0 + w1 * w1 + w2 * w2;
    if (ww <= T * T) return 1;
    const double ub = __builtin_sqrt(ww);
    const double u[3] = {w0 / ub, w1 / ub, w2 / ub};
    const double lb = sd_lower(u, d, n1, A1, n2, A2);
    if (lb > T) return 0;
    if (ub - lb <= 1e-12 * (A1 + A2)) return 1;
    return -1;
}

__device__ __forceinline__ void sd_unit(double v[3])
{
    const double r = __builtin_sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] = v[0] / r;
    v[1] = v[1] / r;
    v[2] = v[2] / r;
}

// Newton's method on the squared distance between the rim points A1 r1 and
// d + A2 r2, rotating r1, r2 by the solved angles (r + s t renormalised,
// t = n x r); stops where the Hessian is not positive definite.
__device__ __noinline__ int sd_newton(const double d[3], const double n1[3], double A1,
                                      const double n2[3], double A2, double T,
                                      const double r1_in[3], const double r2_in[3])
{
    double r1[3] = {r1_in[0], r1_in[1], r1_in[2]}, r2[3] = {r2_in[0], r2_in[1], r2_in[2]};
    for (int j = 0; j < 8; ++j) {
        const double t1[3] = {n1[1] * r1[2] - n1[2] * r1[1], n1[2] * r1[0] - n1[0] * r1[2],
                              n1[0] * r1[1] - n1[1] * r1[0]};
        const double t2[3] = {n2[1] * r2[2] - n2[2] * r2[1], n2[2] * r2[0] - n2[0] * r2[2],
                              n2[0] * r2[1] - n2[1] * r2[0]};
        double w[3];
        for (int a = 0; a < 3; ++a) w[a] = (d[a] + A2 * r2[a]) - A1 * r1[a];
        const double wt1 = w[0] * t1[0] + w[1] * t1[1] + w[2] * t1[2];
        const double wt2 = w[0] * t2[0] + w[1] * t2[1] + w[2] * t2[2];
        const double wr1 = w[0] * r1[0] + w[1] * r1[1] + w[2] * r1[2];
        const double wr2 = w[0] * r2[0] + w[1] * r2[1] + w[2] * r2[2];
        const double tt = t1[0] * t2[0] + t1[1] * t2[1] + t1[2] * t2[2];
        const double g1 = -(A1 * wt1), g2 = A2 * wt2;
        const double h11 = A1 * A1 + A1 * wr1, h22 = A2 * A2 - A2 * wr2, h12 = -(A1 * A2 * tt);
        const double det = h11 * h22 - h12 * h12;
        if (!(h11 > 0.0 && det > 0.0)) return -1;
        const double s1 = -(h22 * g1 - h12 * g2) / det;
        const double s2 = -(h11 * g2 - h12 * g1) / det;
        for (int a = 0; a < 3; ++a) {
            r1[a] = r1[a] + s1 * t1[a];
            r2[a] = r2[a] + s2 * t2[a];
        }
        sd_unit(r1);
        sd_unit(r2);
        double p[3], q[3];
        for (int a = 0; a < 3; ++a) {
            p[a] = A1 * r1[a];
            q[a] = d[a] + A2 * r2[a];
        }
        const int c = sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c;
    }
    return -1;
}

// Is the distance between core disk 1 (centre 0, n1, A1) and core disk 2
// (centre d, n2, A2) at most T?  (The full search runs out of line.)
__device__ __noinline__ bool sd_within_slow(const double d[3], const double n1[3], double A1,
                                            const double n2[3], double A2, double T, double dd)
{
    double u[3];
    if (dd > 0.0) {
        const double r = __builtin_sqrt(dd);
        u[0] = d[0] / r;
        u[1] = d[1] / r;
        u[2] = d[2] / r;
        if (sd_lower(u, d, n1, A1, n2, A2) > T) return false;
    }
    const double h1 = n1[0] * d[0] + n1[1] * d[1] + n1[2] * d[2];
    const double h2 = n2[0] * d[0] + n2[1] * d[1] + n2[2] * d[2];
    for (int a = 0; a < 3; ++a) u[a] = (h1 >= 0.0) ? n1[a] : -n1[a];
    if (sd_lower(u, d, n1, A1, n2, A2) > T) return false;
    for (int a = 0; a < 3; ++a) u[a] = (h2 >= 0.0) ? n2[a] : -n2[a];
    if (sd_lower(u, d, n1, A1, n2, A2) > T) return false;
    double st1[2][3], st2[2][3];
    int ns = 0;
    const double c12 = n2[0] * n1[0] + n2[1] * n1[1] + n2[2] * n1[2];
    double m[3] = {n2[0] - c12 * n1[0], n2[1] - c12 * n1[1], n2[2] - c12 * n1[2]};
    double mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    if (mm > 0.0) {
        const double r = __builtin_sqrt(mm);
        double p[3], x[3], y[3], q[3];
        for (int a = 0; a < 3; ++a) {
            const double e = m[a] / r;
            p[a] = (h2 >= 0.0) ? A1 * e : -(A1 * e);
            x[a] = p[a] - d[a];
        }
        const bool rim = sd_proj(x, n2, A2, y);
        for (int a = 0; a < 3; ++a) q[a] = d[a] + y[a];
        const int c = sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c == 1;
        if (rim) {
            for (int a = 0; a < 3; ++a) {
                st1[ns][a] = p[a];
                st2[ns][a] = y[a];
            }
            sd_unit(st1[ns]);
            sd_unit(st2[ns]);
            ++ns;
        }
    }
    const double c21 = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
    m[0] = n1[0] - c21 * n2[0];
    m[1] = n1[1] - c21 * n2[1];
    m[2] = n1[2] - c21 * n2[2];
    mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    if (mm > 0.0) {
        const double r = __builtin_sqrt(mm);
        double y[3], q[3], p[3];
        for (int a = 0; a < 3; ++a) {
            const double e = m[a] / r;
            y[a] = (h1 >= 0.0) ? -(A2 * e) : A2 * e;
            q[a] = d[a] + y[a];
        }
        const bool rim = sd_proj(q, n1, A1, p);
        const int c = sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c == 1;
        if (rim) {
            for (int a = 0; a < 3; ++a) {
                st1[ns][a] = p[a];
                st2[ns][a] = y[a];
            }
            sd_unit(st1[ns]);
            sd_unit(st2[ns]);
            ++ns;
        }
    }
    double p[3], q[3], x[3], y[3];
    sd_proj(d, n1, A1, p);
    for (int k = 1; k <= 64; ++k) {
        for (int a = 0; a < 3; ++a) x[a] = p[a] - d[a];
        sd_proj(x, n2, A2, y);
        for (int a = 0; a < 3; ++a) q[a] = d[a] + y[a];
        sd_proj(q, n1, A1, p);
        int c = sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c == 1;
        if (k == 6) {
            const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
            const double yy = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
            if (pp > 0.0 && yy > 0.0) {
                double r1[3] = {p[0], p[1], p[2]}, r2[3] = {y[0], y[1], y[2]};
                sd_unit(r1);
                sd_unit(r2);
                c = sd_newton(d, n1, A1, n2, A2, T, r1, r2);
                if (c >= 0) return c == 1;
            }
            for (int j = 0; j < ns; ++j) {
                c = sd_newton(d, n1, A1, n2, A2, T, st1[j], st2[j]);
                if (c >= 0) return c == 1;
            }
        }
    }
    return true;
}

// Spherodisks with centres 0 and d (minimum image of c2 - c1, lower id as
// disk 1), unit normals n1, n2, outer radii a1, a2, half-thicknesses
// tau a: do they overlap when their shells are grown by gap?
__device__ __forceinline__ bool spherodisks_overlap(double dx, double dy, double dz,
                                                    const double n1[3], double a1,
                                                    const double n2[3], double a2, double tau,
                                                    double gap)
{
    const double h1 = tau * a1, h2 = tau * a2;
    const double A1 = a1 - h1, A2 = a2 - h2;
    const double T = (h1 + h2) + gap;
    const double d[3] = {dx, dy, dz};
    const double dd = dx * dx + dy * dy + dz * dz;
    const double R = (A1 + A2) + T;
    if (dd > R * R) return false;
    if (disks_intersect(dx, dy, dz, n1, A1, n2, A2)) return true;
    return sd_within_slow(d, n1, A1, n2, A2, T, dd);
}

// The contact test of two platelets: zero-thickness disks (SD false) or
// spherodisks (SD true; tau = half-thickness / outer radius).
template <bool SD>
__device__ __forceinline__ bool platelets_touch(double dx, double dy, double dz,
                                                const double n1[3], double a1,
                                                const double n2[3], double a2, double tau)
{
    if (SD) return spherodisks_overlap(dx, dy, dz, n1, a1, n2, a2, tau, 0.0);
    return disks_intersect(dx, dy, dz, n1, a1, n2, a2);
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
