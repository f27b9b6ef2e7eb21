/*
 * srm_oracle.c -- plain sequential CPU oracle of the Swelling and Random
 * Migration (SRM) sweep.  TEST INFRASTRUCTURE ONLY: it is the reference the
 * GPU library is checked against and is never called by the library.
 *
 * It computes what the paper's Algorithms 1-6 (Section 2) define, one
 * particle at a time in a sequential order, with the readings listed below.  Positions are stored in particle-id order,
 * array-of-structures pos[3*i + a] (the paper's particle set P with
 * positions r_i); cell lists are Alg. 2's per-cell particle lists, filled in
 * ascending id.
 *
 * Floating point: IEEE binary64, round to nearest, built with
 * -ffp-contract=off -fno-fast-math on x86-64 (SSE2, no x87), so every
 * expression below is evaluated exactly as written, left to right.
 *
 * Readings of the paper (where it is silent or ambiguous):
 *  - swelling (Sec. 2 step a, Alg. 1 step "scale all particles"): additive in
 *    the radius scale s: s' = min(s + c_w * s_target, s_target); R_i = s*rho_i.
 *    The clamp at s_target is the final "minor adjustment" of Sec. 2.
 *  - cell size (Alg. 1): cs = 2.5 * max R' + 2.5 * c_m with the post-swell
 *    radii; per axis m = floor(L/cs) capped at ncap (largest even m with
 *    m^d <= N); the axis is split into N_a = m - (m mod 2) equal cells when
 *    m >= 4, else into one cell.  Even N_a >= 4 makes the 2^d parity colouring
 *    below valid under periodic wrap.
 *  - binning (Alg. 2): c_a = (int)(x_a * (N_a / L_a)), and c_a == N_a -> 0.
 *  - processing order (Alg. 3 "for each particle"): colour phases
 *    g = sum_a (c_a & 1) << a (axes with one cell contribute 0), g ascending;
 *    within a phase cells by ascending linear index c = cx + Nx*(cy + Ny*cz);
 *    within a cell ascending particle id.  Cells of one colour never share a
 *    3^d neighbourhood, so any order of them gives the same result.
 *  - collision test (Alg. 5): contact with any other particle in its current
 *    state, minimum image per axis, squared form q <= (R_i + R_j)^2 (touching
 *    counts as overlap); candidates come from the cells touching the cell of
 *    the tested position.
 *  - unit random vector (Alg. 3): Philox4x32-10 counter-based draws keyed by
 *    the seed, counter (id, sweep, kind<<31 | k<<16 | l<<8 | call, stream);
 *    Marsaglia's rejection method for a uniform point on the sphere (3D) or
 *    a normalised point of the unit disk (2D); no trigonometry.
 *  - shake (Sec. 2 step d, Alg. 1 else-branch): N_k passes over P at P's
 *    radii, re-binning before each pass; s unchanged.
 *  - the sweep counter t advances after every sweep, committed or shaken.
 *  - termination (Sec. 2 step e): s == s_target after a committed sweep.
 *  - thin platelets (Sec. 3.3): zero-thickness disks with a unit normal;
 *    exact disk-disk intersection (chords on the planes' common line); the
 *    centre trial and a normal trial (stream 1, step c_n) are accepted or
 *    rejected together.
 *  - spherodisks (Sec. 3.3 names the platelet model): a particle of
 *    diameter D = 2a and thickness t = thick_ratio * D is the set of points
 *    within h = t/2 of a flat core disk of radius A = a - h (D is the outer
 *    diameter, so the model tends to the zero-thickness disk as t -> 0).
 *    Two spherodisks overlap iff the minimum distance between their core
 *    disks is at most h_i + h_j (touching counts), tested with the lower id
 *    as disk 1.  Volume 2 pi A^2 h + pi^2 A h^2 + 4/3 pi h^3 (Steiner).
 *  - initial configuration (Sec. 2, Alg. 1 "RSA procedure"): classical random
 *    sequential addition of equal particles.  One stream of candidates
 *    k = 0, 1, 2, ... (Philox counters (k_lo, k_hi, call, 2) for the centre,
 *    (k_lo, k_hi, call, 3) for a platelet's normal); a candidate is kept when
 *    it meets none of the particles kept before it (the contact test of
 *    Alg. 5, touching counts) and gets the next particle id.
 */
#include <math.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_EINVAL (-1)
#define O_ENOMEM (-2)
#define O_EOVERLAP (-4)
#define O_ENOTCONV (-5)

#define O_BALL 0
#define O_PLATELET 1
#define O_SPHERODISK 2

#define O_MAIN 0
#define O_SHAKE 1

typedef struct {
    int32_t dim, shape;
    int64_t n;
    double box[3];
    double s_target, c_w, c_m, c_n, thick_ratio;
    int32_t n_k, n_l;
    uint64_t seed;
} o_params;

typedef struct {
    o_params p;
    double *pos;       /* [3n], id order; z unused in 2D */
    double *nrm;       /* [3n] unit normals (platelets) or NULL */
    const double *rho; /* [n] shape radii or NULL (all 1) */
    double s;          /* current radius scale */
    int64_t t;         /* sweep counter */
} o_state;

typedef struct {
    int32_t committed, passes_main, passes_shake, pad;
    int64_t na[3];
    double s_new;
    int64_t n_failed_last;
} o_sweep_info;

typedef struct {
    int64_t na[3];
    double inv_w[3];
    int64_t ncell;
    int64_t *cell;   /* [n] linear cell of each particle */
    int64_t *start;  /* [ncell+1] */
    int64_t *member; /* [n] particle ids grouped by cell, ascending id */
} o_cells;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the  */
/* 4-word multiply/xor bijection with a Weyl key schedule.               */
/* ------------------------------------------------------------------ */
void o_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 32-bit word -> the odd multiple of 2^-32 in (-1, 1): (w - (2^31 - 1/2)) 2^-31
 * (every step exact). */
static double o_sym_uniform(uint32_t w)
{
    return ((double)w - 2147483647.5) * 0x1p-31;
}

/* Random vector of length `len` with uniform direction (Alg. 3, "c_m * Unit
 * Random Vector").  Each Philox call (counter (id, t, kind<<31 | k<<16 |
 * l<<8 | call, stream), key (seed_lo, seed_hi)) gives two attempts (v1, v2)
 * uniform in (-1,1)^2, kept when s = v1^2 + v2^2 < 1.  3D: Marsaglia's
 * point on the sphere (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2s); 2D:
 * (v1, v2) / sqrt(s).  Returns the number of calls used (65 = fallback). */
int o_unitvec(int dim, uint64_t seed, uint64_t id, uint64_t t, uint32_t kind,
              uint32_t k, uint32_t l, uint64_t stream, double len, double v[3])
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t r = 0; r < 64; ++r) {
        uint32_t ctr[4], W[4];
        ctr[0] = (uint32_t)id;
        ctr[1] = (uint32_t)t;
        ctr[2] = (kind << 31) | (k << 16) | (l << 8) | r;
        ctr[3] = (uint32_t)stream;
        o_philox4x32(ctr, key, W);
        for (int a = 0; a < 2; ++a) {
            double v1 = o_sym_uniform(W[2 * a]);
            double v2 = o_sym_uniform(W[2 * a + 1]);
            double s = v1 * v1 + v2 * v2;
            if (s < 1.0) {
                if (dim == 3) {
                    double h = 2.0 * sqrt(1.0 - s);
                    v[0] = (v1 * h) * len;
                    v[1] = (v2 * h) * len;
                    v[2] = (1.0 - 2.0 * s) * len;
                } else {
                    double g = len / sqrt(s);
                    v[0] = v1 * g;
                    v[1] = v2 * g;
                    v[2] = 0.0;
                }
                return (int)r + 1;
            }
        }
    }
    v[0] = len; v[1] = 0.0; v[2] = 0.0;
    return 65;
}

/* Alg. 4: periodic wrapping of one coordinate. */
static double o_wrap(double x, double L)
{
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

/* Minimum-image convention of Alg. 5 for one axis. */
static double o_minimg(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    if (d < -0.5 * L) d += L;
    return d;
}

static double o_radius(const o_state *st, double s, int64_t i)
{
    return st->rho ? s * st->rho[i] : s * 1.0;
}

/* Zero-thickness disk-disk intersection of disk 1 (centre 0, unit normal
 * n1, radius a1) and disk 2 (centre d, n2, a2). */
static int o_disks_meet(const double d[3], const double n1[3], double a1, const double n2[3],
                        double a2)
{
    double dx = d[0], dy = d[1], dz = d[2];
    double dd = dx * dx + dy * dy + dz * dz;
    double sa = a1 + a2;
    if (dd > sa * sa) return 0;
    /* u = n1 x n2: direction of the planes' common line */
    double ux = n1[1] * n2[2] - n1[2] * n2[1];
    double uy = n1[2] * n2[0] - n1[0] * n2[2];
    double uz = n1[0] * n2[1] - n1[1] * n2[0];
    double uu = ux * ux + uy * uy + uz * uz;
    if (uu == 0.0) {
        /* parallel planes: intersect only when coplanar (circle test) */
        double hn = n1[0] * dx + n1[1] * dy + n1[2] * dz;
        return hn == 0.0;
    }
    /* foot p of centre 1 on the common line: p = (u x n1) * (h / uu) */
    double h = n2[0] * dx + n2[1] * dy + n2[2] * dz;
    double wx = uy * n1[2] - uz * n1[1];
    double wy = uz * n1[0] - ux * n1[2];
    double wz = ux * n1[1] - uy * n1[0];
    double f = h / uu;
    double px = wx * f, py = wy * f, pz = wz * f;
    double A = a1 * a1 - (px * px + py * py + pz * pz);
    if (A < 0.0) return 0;
    /* foot of centre 2: p + t0 u */
    double ex = dx - px, ey = dy - py, ez = dz - pz;
    double t0 = (ex * ux + ey * uy + ez * uz) / uu;
    double B = a2 * a2 - ((ex * ex + ey * ey + ez * ez) - (t0 * t0) * uu);
    if (B < 0.0) return 0;
    /* chords [-sqrt(A/uu), sqrt(A/uu)] and t0 +- sqrt(B/uu) overlap */
    double Ap = A / uu, Bp = B / uu, C = t0 * t0;
    double D = (C - Ap) - Bp;
    if (D <= 0.0) return 1;
    return D * D <= (4.0 * Ap) * Bp;
}

/* The same test for disks at c1 and c2 (minimum image of c2 - c1); callers
 * pass the lower particle id as disk 1. */
int o_disks_intersect(const double c1[3], const double n1[3], double a1,
                      const double c2[3], const double n2[3], double a2,
                      const double box[3])
{
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = o_minimg(c2[a] - c1[a], box[a]);
    return o_disks_meet(d, n1, a1, n2, a2);
}

/* ---- spherodisks: is the distance between two core disks at most T? ----
 * Core disk 1 has centre 0, unit normal n1, radius A1; core disk 2 has
 * centre d, n2, A2.  The decision rests on two kinds of certificate:
 *  - a pair of points p on disk 1 and q on disk 2 with |q - p| <= T proves
 *    overlap;
 *  - a unit direction u with L(u) = u.d - A1 |u x n1| - A2 |u x n2| > T
 *    proves separation: the projections of the two disks on u are at
 *    least L(u) apart (A |u x n| is a disk's half-extent along u), so every
 *    pair of points is.
 * At the closest pair (p*, q*) the direction (q* - p*)/|q* - p*| gives
 * L = |q* - p*|, so the certificates meet at the true distance.  Pairs
 * come from (in order) the zero-thickness intersection test, the point of
 * each rim nearest the other disk's plane, alternating projections between
 * the disks (which converge to a closest pair of two disjoint convex sets),
 * and Newton's method on the two rim angles started from those pairs.
 * Where no certificate decides -- the distance lies within 1e-12 (A1 + A2)
 * of T, or the iterations run out -- the pair counts as overlapping, the
 * conservative side for admissibility. */
static double o_sd_lower(const double u[3], const double d[3], const double n1[3], double A1,
                         const double n2[3], double A2)
{
    double x0 = u[1] * n1[2] - u[2] * n1[1];
    double x1 = u[2] * n1[0] - u[0] * n1[2];
    double x2 = u[0] * n1[1] - u[1] * n1[0];
    double y0 = u[1] * n2[2] - u[2] * n2[1];
    double y1 = u[2] * n2[0] - u[0] * n2[2];
    double y2 = u[0] * n2[1] - u[1] * n2[0];
    double e1 = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
    double e2 = sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    double ud = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    return (ud - A1 * e1) - A2 * e2;
}

/* Nearest point y of the disk (centre 0, unit normal n, radius A) to x;
 * returns 1 when y lies on the rim. */
static int o_sd_proj(const double x[3], const double n[3], double A, double y[3])
{
    double h = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    y[0] = x[0] - h * n[0];
    y[1] = x[1] - h * n[1];
    y[2] = x[2] - h * n[2];
    double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    if (r2 <= A * A) return 0;
    double f = A / sqrt(r2);
    y[0] = y[0] * f;
    y[1] = y[1] * f;
    y[2] = y[2] * f;
    return 1;
}

#define O_SD_BAND 1e-12

/* 1: overlap, 0: separated, -1: the pair (p, q) decides nothing. */
static int o_sd_certify(const double p[3], const double q[3], const double d[3],
                        const double n1[3], double A1, const double n2[3], double A2, double T)
{
    double w0 = q[0] - p[0], w1 = q[1] - p[1], w2 = q[2] - p[2];
    double ww = w0 * w0 + w1 * w1 + w2 * w2;
    if (ww <= T * T) return 1;
    double ub = sqrt(ww);
    double u[3] = {w0 / ub, w1 / ub, w2 / ub};
    double lb = o_sd_lower(u, d, n1, A1, n2, A2);
    if (lb > T) return 0;
    if (ub - lb <= O_SD_BAND * (A1 + A2)) return 1;
    return -1;
}

static void o_sd_unit(double v[3])
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] = v[0] / r;
    v[1] = v[1] / r;
    v[2] = v[2] / r;
}

/* Newton's method on the squared distance between the rim points A1 r1
 * and d + A2 r2 (r1, r2 unit vectors in the disks' planes), each step
 * rotating r1, r2 by the solved angles (r + s t, renormalised, t = n x r).
 * Stops where the Hessian is not positive definite. */
static int o_sd_newton(const double d[3], const double n1[3], double A1, const double n2[3],
                       double A2, double T, const double r1_in[3], const double r2_in[3])
{
    double r1[3] = {r1_in[0], r1_in[1], r1_in[2]}, r2[3] = {r2_in[0], r2_in[1], r2_in[2]};
    for (int j = 0; j < 8; ++j) {
        double t1[3] = {n1[1] * r1[2] - n1[2] * r1[1], n1[2] * r1[0] - n1[0] * r1[2],
                        n1[0] * r1[1] - n1[1] * r1[0]};
        double t2[3] = {n2[1] * r2[2] - n2[2] * r2[1], n2[2] * r2[0] - n2[0] * r2[2],
                        n2[0] * r2[1] - n2[1] * r2[0]};
        double w[3];
        for (int a = 0; a < 3; ++a) w[a] = (d[a] + A2 * r2[a]) - A1 * r1[a];
        double wt1 = w[0] * t1[0] + w[1] * t1[1] + w[2] * t1[2];
        double wt2 = w[0] * t2[0] + w[1] * t2[1] + w[2] * t2[2];
        double wr1 = w[0] * r1[0] + w[1] * r1[1] + w[2] * r1[2];
        double wr2 = w[0] * r2[0] + w[1] * r2[1] + w[2] * r2[2];
        double tt = t1[0] * t2[0] + t1[1] * t2[1] + t1[2] * t2[2];
        /* half the gradient and Hessian of |w|^2 in the two rim angles */
        double g1 = -(A1 * wt1), g2 = A2 * wt2;
        double h11 = A1 * A1 + A1 * wr1, h22 = A2 * A2 - A2 * wr2, h12 = -(A1 * A2 * tt);
        double det = h11 * h22 - h12 * h12;
        if (!(h11 > 0.0 && det > 0.0)) return -1;
        double s1 = -(h22 * g1 - h12 * g2) / det;
        double s2 = -(h11 * g2 - h12 * g1) / det;
        for (int a = 0; a < 3; ++a) {
            r1[a] = r1[a] + s1 * t1[a];
            r2[a] = r2[a] + s2 * t2[a];
        }
        o_sd_unit(r1);
        o_sd_unit(r2);
        double p[3], q[3];
        for (int a = 0; a < 3; ++a) {
            p[a] = A1 * r1[a];
            q[a] = d[a] + A2 * r2[a];
        }
        int c = o_sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c;
    }
    return -1;
}

/* Is the minimum distance between core disk 1 (centre 0, n1, A1) and core
 * disk 2 (centre d, n2, A2) at most T (T >= 0)? */
int o_sd_within(const double d[3], const double n1[3], double A1, const double n2[3], double A2,
                double T)
{
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double R = (A1 + A2) + T;
    if (dd > R * R) return 0;
    if (o_disks_meet(d, n1, A1, n2, A2)) return 1;
    /* separating directions: the centre line and both normals */
    double u[3];
    if (dd > 0.0) {
        double r = sqrt(dd);
        u[0] = d[0] / r;
        u[1] = d[1] / r;
        u[2] = d[2] / r;
        if (o_sd_lower(u, d, n1, A1, n2, A2) > T) return 0;
    }
    double h1 = n1[0] * d[0] + n1[1] * d[1] + n1[2] * d[2];
    double h2 = n2[0] * d[0] + n2[1] * d[1] + n2[2] * d[2];
    for (int a = 0; a < 3; ++a) u[a] = (h1 >= 0.0) ? n1[a] : -n1[a];
    if (o_sd_lower(u, d, n1, A1, n2, A2) > T) return 0;
    for (int a = 0; a < 3; ++a) u[a] = (h2 >= 0.0) ? n2[a] : -n2[a];
    if (o_sd_lower(u, d, n1, A1, n2, A2) > T) return 0;
    /* the point of each rim nearest the other disk's plane; where its
     * projection leaves the other disk, the pair starts a Newton run */
    double st1[2][3], st2[2][3];
    int ns = 0;
    double c12 = n2[0] * n1[0] + n2[1] * n1[1] + n2[2] * n1[2];
    double m[3] = {n2[0] - c12 * n1[0], n2[1] - c12 * n1[1], n2[2] - c12 * n1[2]};
    double mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    if (mm > 0.0) {
        double r = sqrt(mm), p[3], x[3], y[3], q[3];
        for (int a = 0; a < 3; ++a) {
            double e = m[a] / r;
            p[a] = (h2 >= 0.0) ? A1 * e : -(A1 * e);
            x[a] = p[a] - d[a];
        }
        int rim = o_sd_proj(x, n2, A2, y);
        for (int a = 0; a < 3; ++a) q[a] = d[a] + y[a];
        int c = o_sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c;
        if (rim) {
            for (int a = 0; a < 3; ++a) {
                st1[ns][a] = p[a];
                st2[ns][a] = y[a];
            }
            o_sd_unit(st1[ns]);
            o_sd_unit(st2[ns]);
            ++ns;
        }
    }
    double c21 = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
    m[0] = n1[0] - c21 * n2[0];
    m[1] = n1[1] - c21 * n2[1];
    m[2] = n1[2] - c21 * n2[2];
    mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    if (mm > 0.0) {
        double r = sqrt(mm), y[3], q[3], p[3];
        for (int a = 0; a < 3; ++a) {
            double e = m[a] / r;
            y[a] = (h1 >= 0.0) ? -(A2 * e) : A2 * e;
            q[a] = d[a] + y[a];
        }
        int rim = o_sd_proj(q, n1, A1, p);
        int c = o_sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c;
        if (rim) {
            for (int a = 0; a < 3; ++a) {
                st1[ns][a] = p[a];
                st2[ns][a] = y[a];
            }
            o_sd_unit(st1[ns]);
            o_sd_unit(st2[ns]);
            ++ns;
        }
    }
    /* alternating projections from the point of disk 1 nearest disk 2's
     * centre; after six rounds, Newton from the current pair and from the
     * rim starts above */
    double p[3], q[3], x[3], y[3];
    o_sd_proj(d, n1, A1, p);
    for (int k = 1; k <= 64; ++k) {
        for (int a = 0; a < 3; ++a) x[a] = p[a] - d[a];
        o_sd_proj(x, n2, A2, y);
        for (int a = 0; a < 3; ++a) q[a] = d[a] + y[a];
        o_sd_proj(q, n1, A1, p);
        int c = o_sd_certify(p, q, d, n1, A1, n2, A2, T);
        if (c >= 0) return c;
        if (k == 6) {
            double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
            double yy = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
            if (pp > 0.0 && yy > 0.0) {
                double r1[3] = {p[0], p[1], p[2]}, r2[3] = {y[0], y[1], y[2]};
                o_sd_unit(r1);
                o_sd_unit(r2);
                c = o_sd_newton(d, n1, A1, n2, A2, T, r1, r2);
                if (c >= 0) return c;
            }
            for (int j = 0; j < ns; ++j) {
                c = o_sd_newton(d, n1, A1, n2, A2, T, st1[j], st2[j]);
                if (c >= 0) return c;
            }
        }
    }
    return 1;
}

/* Spherodisks at c1 and c2 (outer radii a1, a2; half-thicknesses
 * h = thick_ratio * a): do they overlap?  Lower particle id as disk 1. */
int o_spherodisks_overlap(const double c1[3], const double n1[3], double a1,
                          const double c2[3], const double n2[3], double a2,
                          double thick_ratio, double gap, const double box[3])
{
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = o_minimg(c2[a] - c1[a], box[a]);
    double h1 = thick_ratio * a1, h2 = thick_ratio * a2;
    return o_sd_within(d, n1, a1 - h1, n2, a2 - h2, (h1 + h2) + gap);
}

/* ------------------------------------------------------------------ */
/* Cells (Alg. 1 cell size, Alg. 2 build cell list).                   */
/* ------------------------------------------------------------------ */
static int64_t o_ncap(int dim, int64_t n)
{
    int64_t m = 0;
    for (;;) {
        int64_t c = m + 2, pw = 1;
        for (int a = 0; a < dim; ++a) pw *= c;
        if (pw > n) break;
        m = c;
    }
    return m;
}

void o_grid(const o_params *p, double rmax, int64_t na[3], double inv_w[3])
{
    double cs = 2.5 * rmax + 2.5 * p->c_m;
    int64_t ncap = o_ncap(p->dim, p->n);
    for (int a = 0; a < 3; ++a) {
        if (a >= p->dim) { na[a] = 1; inv_w[a] = 1.0 / p->box[a]; continue; }
        int64_t m;
        double q = (cs > 0.0) ? p->box[a] / cs : 0.0;
        if (!(cs > 0.0) || q >= (double)ncap) m = ncap;
        else m = (int64_t)q;
        na[a] = (m >= 4) ? m - (m & 1) : 1;
        inv_w[a] = (double)na[a] / p->box[a];
    }
}

static void o_cell_coords(const o_cells *g, const double x[3], int dim, int64_t c[3])
{
    for (int a = 0; a < 3; ++a) {
        if (a >= dim) { c[a] = 0; continue; }
        int64_t ca = (int64_t)(x[a] * g->inv_w[a]);
        if (ca == g->na[a]) ca = 0;
        c[a] = ca;
    }
}

static int64_t o_linear(const o_cells *g, const int64_t c[3])
{
    return c[0] + g->na[0] * (c[1] + g->na[1] * c[2]);
}

static void o_cells_free(o_cells *g)
{
    free(g->cell); free(g->start); free(g->member);
    g->cell = g->start = g->member = NULL;
}

static int o_cells_build(o_cells *g, const o_params *p, const int64_t na[3],
                         const double inv_w[3], const double *pos)
{
    int64_t n = p->n;
    for (int a = 0; a < 3; ++a) { g->na[a] = na[a]; g->inv_w[a] = inv_w[a]; }
    g->ncell = na[0] * na[1] * na[2];
    g->cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    g->start = (int64_t *)calloc((size_t)g->ncell + 1, sizeof(int64_t));
    g->member = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!g->cell || !g->start || !g->member) { o_cells_free(g); return O_ENOMEM; }
    /* Alg. 2: for each particle q (ascending id): cells[c].Add(q) */
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        o_cell_coords(g, &pos[3 * i], p->dim, c);
        g->cell[i] = o_linear(g, c);
        g->start[g->cell[i] + 1] += 1;
    }
    for (int64_t c = 0; c < g->ncell; ++c) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->ncell > 0 ? g->ncell : 1));
    if (!fill) { o_cells_free(g); return O_ENOMEM; }
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)g->ncell);
    for (int64_t i = 0; i < n; ++i) g->member[fill[g->cell[i]]++] = i;
    free(fill);
    return O_OK;
}

/* Cell assignment only (Alg. 2 lines computing c_x, c_y[, c_z]). */
int o_bin(const o_params *p, const int64_t na[3], const double inv_w[3],
          const double *pos, int64_t *cell_out)
{
    o_cells g;
    for (int a = 0; a < 3; ++a) { g.na[a] = na[a]; g.inv_w[a] = inv_w[a]; }
    for (int64_t i = 0; i < p->n; ++i) {
        int64_t c[3];
        o_cell_coords(&g, &pos[3 * i], p->dim, c);
        cell_out[i] = o_linear(&g, c);
    }
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Alg. 5: does particle i, tested at position y, meet another particle?  */
/* ------------------------------------------------------------------ */
/* Contact of particle i at (y, normal ny) with particle j in its current
 * state.  Balls: the minimum-image squared centre distance is at most
 * (R_i + R_j)^2 (touching counts).  Thin disks: they intersect, tested with
 * the lower particle id as disk 1 so that both orders of a pair agree. */
static int o_contact(const o_state *st, int64_t i, const double y[3], const double ny[3],
                     int64_t j, double s)
{
    const o_params *p = &st->p;
    const double *xj = &st->pos[3 * j];
    double Ri = o_radius(st, s, i), Rj = o_radius(st, s, j);
    if (p->shape == O_PLATELET) {
        const double *nj = &st->nrm[3 * j];
        return (i < j) ? o_disks_intersect(y, ny, Ri, xj, nj, Rj, p->box)
                       : o_disks_intersect(xj, nj, Rj, y, ny, Ri, p->box);
    }
    if (p->shape == O_SPHERODISK) {
        const double *nj = &st->nrm[3 * j];
        return (i < j) ? o_spherodisks_overlap(y, ny, Ri, xj, nj, Rj, p->thick_ratio, 0.0, p->box)
                       : o_spherodisks_overlap(xj, nj, Rj, y, ny, Ri, p->thick_ratio, 0.0, p->box);
    }
    double d0 = o_minimg(y[0] - xj[0], p->box[0]);
    double d1 = o_minimg(y[1] - xj[1], p->box[1]);
    double q = d0 * d0 + d1 * d1;
    if (p->dim == 3) {
        double d2 = o_minimg(y[2] - xj[2], p->box[2]);
        q = q + d2 * d2;
    }
    double sig = Ri + Rj;
    return q <= sig * sig;
}

/* Linear indices of the cells that touch cell c (c itself included) under
 * periodic wrap: one cell either side along every axis split into cells, a
 * single cell along an axis that is not split. */
static int o_touching_cells(const o_cells *g, const int64_t c[3], int64_t out[27])
{
    int count = 0;
    int64_t span[3];
    for (int a = 0; a < 3; ++a) span[a] = (g->na[a] > 1) ? 3 : 1;
    for (int64_t k = 0; k < span[0] * span[1] * span[2]; ++k) {
        int64_t off[3] = {k % span[0], (k / span[0]) % span[1], k / (span[0] * span[1])};
        int64_t nc[3];
        for (int a = 0; a < 3; ++a) {
            int64_t shift = (span[a] == 3) ? off[a] - 1 : 0;
            nc[a] = (c[a] + shift + g->na[a]) % g->na[a];
        }
        out[count++] = o_linear(g, nc);
    }
    return count;
}

/* Particle i at y collides when it is in contact with any other particle.
 * Every particle close enough to touch lies in a cell touching y's cell (the
 * cell edge covers the largest contact distance), so the lists of those
 * cells hold every candidate. */
static int o_collides(const o_state *st, const o_cells *g, int64_t i,
                      const double y[3], const double ny[3], double s)
{
    int64_t c[3], cells[27];
    o_cell_coords(g, y, st->p.dim, c);
    int count = o_touching_cells(g, c, cells);
    for (int b = 0; b < count; ++b) {
        for (int64_t m = g->start[cells[b]]; m < g->start[cells[b] + 1]; ++m) {
            int64_t j = g->member[m];
            if (j != i && o_contact(st, i, y, ny, j, s)) return 1;
        }
    }
    return 0;
}

/* Alg. 6: is there any colliding particle (lists from the last binning). */
static int o_any_collision(const o_state *st, const o_cells *g, double s)
{
    for (int64_t i = 0; i < st->p.n; ++i) {
        const double *nyi = st->nrm ? &st->nrm[3 * i] : NULL;
        if (o_collides(st, g, i, &st->pos[3 * i], nyi, s)) return 1;
    }
    return 0;
}

static int o_colour_of(const o_cells *g, int64_t cl, int dim)
{
    int64_t c0 = cl % g->na[0];
    int64_t c1 = (cl / g->na[0]) % g->na[1];
    int64_t c2 = cl / (g->na[0] * g->na[1]);
    int64_t c[3] = {c0, c1, c2};
    int col = 0;
    for (int a = 0; a < dim; ++a)
        if (g->na[a] >= 4) col |= (int)(c[a] & 1) << a;
    return col;
}

/* One trial displacement of particle i: y = wrap(old + v), and for platelets
 * the trial normal m/|m| with m = n_old + w. */
static void o_trial(const o_state *st, int64_t i, const double old[3], const double nold[3],
                    uint32_t kind, uint32_t k, uint32_t l, double y[3], double ny[3])
{
    const o_params *p = &st->p;
    double v[3];
    o_unitvec(p->dim, p->seed, (uint64_t)i, (uint64_t)st->t, kind, k, l, 0, p->c_m, v);
    for (int a = 0; a < 3; ++a) {
        if (a < p->dim) y[a] = o_wrap(old[a] + v[a], p->box[a]);
        else y[a] = old[a];
    }
    if (p->shape == O_PLATELET || p->shape == O_SPHERODISK) {
        double w[3];
        o_unitvec(3, p->seed, (uint64_t)i, (uint64_t)st->t, kind, k, l, 1, p->c_n, w);
        double m0 = nold[0] + w[0], m1 = nold[1] + w[1], m2 = nold[2] + w[2];
        double mm = m0 * m0 + m1 * m1 + m2 * m2;
        double inv = 1.0 / sqrt(mm);
        ny[0] = m0 * inv; ny[1] = m1 * inv; ny[2] = m2 * inv;
    }
}

/* Alg. 3 over the colour schedule: one migration pass.  `g` are the lists
 * built at the start of the pass (Alg. 1 fills cells before each move).
 * `mask` (optional, per linear cell) restricts the pass to a set of cells. */
static void o_move(o_state *st, const o_cells *g, double s, uint32_t kind, uint32_t k,
                   uint8_t *acc, const uint8_t *mask)
{
    const o_params *p = &st->p;
    int ncol = 1 << p->dim;
    for (int col = 0; col < ncol; ++col) {
        for (int64_t cl = 0; cl < g->ncell; ++cl) {
            if (o_colour_of(g, cl, p->dim) != col) continue;
            if (mask && !mask[cl]) continue;
            for (int64_t m = g->start[cl]; m < g->start[cl + 1]; ++m) {
                int64_t i = g->member[m];
                double *q = &st->pos[3 * i];
                double *nq = st->nrm ? &st->nrm[3 * i] : NULL;
                double old[3] = {q[0], q[1], q[2]};
                double nold[3] = {0.0, 0.0, 0.0};
                if (nq) { nold[0] = nq[0]; nold[1] = nq[1]; nold[2] = nq[2]; }
                uint8_t code = 0;
                for (int32_t l = 1; l <= p->n_l; ++l) {
                    double y[3], ny[3] = {0.0, 0.0, 0.0};
                    o_trial(st, i, old, nold, kind, k, (uint32_t)l, y, ny);
                    if (!o_collides(st, g, i, y, ny, s)) {
                        q[0] = y[0]; q[1] = y[1]; q[2] = y[2];
                        if (nq) { nq[0] = ny[0]; nq[1] = ny[1]; nq[2] = ny[2]; }
                        code = (uint8_t)l;
                        break;
                    }
                    /* q = q_old: the stored position was never changed */
                }
                if (acc) acc[i] = code;
            }
        }
    }
}

/* Fill cells (Alg. 2) then move (Alg. 3) once: one pass at radius scale s. */
int o_pass(o_state *st, const int64_t na[3], const double inv_w[3], double s,
           uint32_t kind, uint32_t k, uint8_t *acc, const uint8_t *mask, int32_t *overlap)
{
    o_cells g;
    int rc = o_cells_build(&g, &st->p, na, inv_w, st->pos);
    if (rc) return rc;
    o_move(st, &g, s, kind, k, acc, mask);
    if (overlap) *overlap = o_any_collision(st, &g, s);
    o_cells_free(&g);
    return O_OK;
}

/* Alg. 6 on a freshly built cell list. */
int o_overlap(const o_state *st, const int64_t na[3], const double inv_w[3], double s,
              int32_t *overlap)
{
    o_cells g;
    int rc = o_cells_build(&g, &st->p, na, inv_w, st->pos);
    if (rc) return rc;
    *overlap = o_any_collision(st, &g, s);
    o_cells_free(&g);
    return O_OK;
}

double o_rho_max(const o_state *st)
{
    if (!st->rho) return 1.0;
    double m = 0.0;
    for (int64_t i = 0; i < st->p.n; ++i) if (st->rho[i] > m) m = st->rho[i];
    return m;
}

/* Radius scale after one swelling step, clamped at s_stop (the target
 * scale, or an intermediate one of a staged run). */
static double o_swell_to(const o_params *p, double s, double s_stop)
{
    double ds = p->c_w * p->s_target;
    double s1 = s + ds;
    return (s1 < s_stop) ? s1 : s_stop;
}

double o_swell(const o_params *p, double s)
{
    return o_swell_to(p, s, p->s_target);
}

/* ------------------------------------------------------------------ */
/* Alg. 1: one iteration of the main loop (one sweep).                 */
/* ------------------------------------------------------------------ */
static int o_sweep_to(o_state *st, double s_stop, o_sweep_info *info, uint8_t *acc_last)
{
    const o_params *p = &st->p;
    int64_t n = p->n;
    double s1 = o_swell_to(p, st->s, s_stop);
    int64_t na[3]; double inv_w[3];
    o_grid(p, s1 * o_rho_max(st), na, inv_w);
    size_t bytes = sizeof(double) * 3 * (size_t)(n > 0 ? n : 1);
    /* Q = P */
    double *qpos = (double *)malloc(bytes);
    double *qnrm = st->nrm ? (double *)malloc(bytes) : NULL;
    uint8_t *acc = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!qpos || !acc || (st->nrm && !qnrm)) { free(qpos); free(qnrm); free(acc); return O_ENOMEM; }
    memcpy(qpos, st->pos, bytes);
    if (qnrm) memcpy(qnrm, st->nrm, bytes);
    o_state q = *st;
    q.pos = qpos; q.nrm = qnrm;
    int collision = 1;
    int32_t passes_main = 0, passes_shake = 0;
    for (int32_t k = 1; k <= p->n_k; ++k) {
        int32_t ov = 1;
        int rc = o_pass(&q, na, inv_w, s1, O_MAIN, (uint32_t)k, acc, NULL, &ov);
        if (rc) { free(qpos); free(qnrm); free(acc); return rc; }
        passes_main++;
        collision = ov;
        if (!collision) break;
    }
    int64_t nfail = 0;
    if (passes_main > 0) for (int64_t i = 0; i < n; ++i) nfail += (acc[i] == 0);
    if (!collision) {
        memcpy(st->pos, qpos, bytes);      /* P = Q */
        if (qnrm) memcpy(st->nrm, qnrm, bytes);
        st->s = s1;                         /* update volume fraction */
        if (acc_last) memcpy(acc_last, acc, (size_t)n);
    } else {
        /* shake: N_k passes over P at P's radii, re-binned before each */
        for (int32_t j = 1; j <= p->n_k; ++j) {
            int rc = o_pass(st, na, inv_w, st->s, O_SHAKE, (uint32_t)j, acc, NULL, NULL);
            if (rc) { free(qpos); free(qnrm); free(acc); return rc; }
            passes_shake++;
        }
        if (acc_last) memcpy(acc_last, acc, (size_t)n);
    }
    st->t += 1;
    if (info) {
        info->committed = !collision;
        info->passes_main = passes_main;
        info->passes_shake = passes_shake;
        for (int a = 0; a < 3; ++a) info->na[a] = na[a];
        info->s_new = st->s;
        info->n_failed_last = nfail;
    }
    free(qpos); free(qnrm); free(acc);
    return O_OK;
}

int o_sweep(o_state *st, o_sweep_info *info, uint8_t *acc_last)
{
    return o_sweep_to(st, st->p.s_target, info, acc_last);
}

/* Alg. 1 while loop: sweep until s == s_stop (swelling clamped there) or
 * max_sweeps sweeps.  s_stop is the target scale, or a smaller one for a
 * stage of a staged run. */
int o_run_to(o_state *st, double s_stop, int32_t max_sweeps, int64_t *sweeps_out,
             int64_t *passes_out)
{
    int64_t sweeps = 0, passes = 0;
    while (st->s < s_stop) {
        if (sweeps >= max_sweeps) {
            if (sweeps_out) *sweeps_out = sweeps;
            if (passes_out) *passes_out = passes;
            return O_ENOTCONV;
        }
        o_sweep_info info;
        int rc = o_sweep_to(st, s_stop, &info, NULL);
        if (rc) return rc;
        sweeps++;
        passes += info.passes_main + info.passes_shake;
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (passes_out) *passes_out = passes;
    return O_OK;
}

int o_run(o_state *st, int32_t max_sweeps, int64_t *sweeps_out, int64_t *passes_out)
{
    return o_run_to(st, st->p.s_target, max_sweeps, sweeps_out, passes_out);
}

/* ------------------------------------------------------------------ */
/* Random sequential addition (Sec. 2: the non-overlapping start at f0). */
/* ------------------------------------------------------------------ */
/* 53-bit uniform in [0, 1) from two words: the top 27 bits of the first and
 * the top 26 of the second, ((w_a >> 5) 2^26 + (w_b >> 6)) 2^-53 (exact). */
static double o_u53(uint32_t wa, uint32_t wb)
{
    return ((double)(wa >> 5) * 67108864.0 + (double)(wb >> 6)) * 0x1p-53;
}

/* Candidate k of the RSA stream: centre u_a * L_a per axis, axes 0 and 1 from
 * the words of call 0 and axis 2 from the first two words of call 1 (counter
 * (k_lo, k_hi, call, 2)); a product that rounds up to L_a is folded to 0.
 * Platelets: unit normal from the sphere-point method of Alg. 3's random
 * vector with length 1, counter (k_lo, k_hi, call, 3). */
void o_rsa_candidate(int dim, int shape, const double box[3], uint64_t seed, uint64_t k,
                     double x[3], double nrm[3])
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), 0u, 2u}, W[4];
    o_philox4x32(ctr, key, W);
    x[0] = o_u53(W[0], W[1]) * box[0];
    x[1] = o_u53(W[2], W[3]) * box[1];
    x[2] = 0.0;
    if (dim == 3) {
        ctr[2] = 1u;
        o_philox4x32(ctr, key, W);
        x[2] = o_u53(W[0], W[1]) * box[2];
    }
    for (int a = 0; a < dim; ++a)
        if (x[a] >= box[a]) x[a] = 0.0;
    if (shape == O_PLATELET)
        o_unitvec(3, seed, (uint32_t)k, (uint32_t)(k >> 32), 0, 0, 0, 3, 1.0, nrm);
}

/* Classical RSA of n equal particles (balls of radius `radius`, or platelets
 * of radius `radius`): candidates are drawn in stream order and kept when
 * they meet no particle kept earlier (balls: q <= (R + R)^2 with the
 * minimum image of candidate - kept; platelets: the disk test with the kept
 * particle as disk 1).  Kept candidates are numbered 0, 1, ... in the order
 * kept; pos/nrm are [3n] rows (z = 0 in 2D), src[i] (nullable) is the
 * candidate index of particle i.  *drawn = candidates drawn (the index of
 * the last kept one plus 1), *placed = particles placed.  Returns O_ENOTCONV
 * when max_candidates are drawn before n are placed. */
int o_rsa(int dim, int shape, int64_t n, const double box[3], double radius, uint64_t seed,
          int64_t max_candidates, double *pos, double *nrm, int64_t *src, int64_t *drawn,
          int64_t *placed)
{
    if ((dim != 2 && dim != 3) || (shape != O_BALL && shape != O_PLATELET) ||
        (shape == O_PLATELET && dim != 3) || n < 0 || !(radius >= 0.0) || isinf(radius))
        return O_EINVAL;
    for (int a = 0; a < dim; ++a)
        if (!(box[a] > 0.0) || isinf(box[a])) return O_EINVAL;
    const double sig = radius + radius;
    int64_t kept = 0, k = 0;
    while (kept < n) {
        if (k >= max_candidates) {
            *drawn = k;
            *placed = kept;
            return O_ENOTCONV;
        }
        double x[3], m[3] = {0.0, 0.0, 0.0};
        o_rsa_candidate(dim, shape, box, seed, (uint64_t)k, x, m);
        int hit = 0;
        for (int64_t j = 0; j < kept && !hit; ++j) {
            const double *y = &pos[3 * j];
            if (shape == O_BALL) {
                double d0 = o_minimg(x[0] - y[0], box[0]);
                double d1 = o_minimg(x[1] - y[1], box[1]);
                double q = d0 * d0 + d1 * d1;
                if (dim == 3) {
                    double d2 = o_minimg(x[2] - y[2], box[2]);
                    q = q + d2 * d2;
                }
                hit = q <= sig * sig;
            } else {
                hit = o_disks_intersect(y, &nrm[3 * j], radius, x, m, radius, box);
            }
        }
        if (!hit) {
            for (int a = 0; a < 3; ++a) {
                pos[3 * kept + a] = x[a];
                if (nrm) nrm[3 * kept + a] = m[a];
            }
            if (src) src[kept] = k;
            kept++;
        }
        k++;
    }
    *drawn = k;
    *placed = kept;
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Brute-force references (all pairs, O(N^2)).                        */
/* ------------------------------------------------------------------ */
static double o_pair_q(const o_state *st, int64_t i, int64_t j)
{
    const o_params *p = &st->p;
    const double *xi = &st->pos[3 * i], *xj = &st->pos[3 * j];
    double d0 = o_minimg(xi[0] - xj[0], p->box[0]);
    double d1 = o_minimg(xi[1] - xj[1], p->box[1]);
    double q = d0 * d0 + d1 * d1;
    if (p->dim == 3) {
        double d2 = o_minimg(xi[2] - xj[2], p->box[2]);
        q = q + d2 * d2;
    }
    return q;
}

/* Pairs i<j whose shapes, grown by `gap` ((R_i + R_j) + gap for balls; radii
 * a + gap/2 for zero-thickness platelets; core-disk distance at most
 * h_i + h_j + gap for spherodisks, i.e. shells of thickness gap/2 around
 * each surface), overlap or touch; written sorted by (i, j).
 * Returns the total count (which may exceed cap; only cap pairs written). */
int64_t o_pairs_brute(const o_state *st, double s, double gap, int64_t cap, int32_t *ij)
{
    const o_params *p = &st->p;
    int64_t cnt = 0;
    for (int64_t i = 0; i < p->n; ++i) {
        for (int64_t j = i + 1; j < p->n; ++j) {
            int hit;
            if (p->shape == O_PLATELET) {
                double ai = o_radius(st, s, i) + 0.5 * gap, aj = o_radius(st, s, j) + 0.5 * gap;
                hit = o_disks_intersect(&st->pos[3 * i], &st->nrm[3 * i], ai,
                                        &st->pos[3 * j], &st->nrm[3 * j], aj, p->box);
            } else if (p->shape == O_SPHERODISK) {
                hit = o_spherodisks_overlap(&st->pos[3 * i], &st->nrm[3 * i], o_radius(st, s, i),
                                            &st->pos[3 * j], &st->nrm[3 * j], o_radius(st, s, j),
                                            p->thick_ratio, gap, p->box);
            } else {
                double sig = (o_radius(st, s, i) + o_radius(st, s, j)) + gap;
                hit = o_pair_q(st, i, j) <= sig * sig;
            }
            if (hit) {
                if (cnt < cap) { ij[2 * cnt] = (int32_t)i; ij[2 * cnt + 1] = (int32_t)j; }
                cnt++;
            }
        }
    }
    return cnt;
}

/* Hard core - soft shell percolation (Sec. 3.3): particles are bonded when
 * they overlap after growing by `gap` (the o_pairs_brute predicate); a
 * cluster percolates along axis a when it wraps around the periodic box
 * along a.  Union-find in which every particle keeps its periodic image
 * relative to its parent: a bond i-j whose nearest image of j is x_j + s L
 * (s_a = +1 when x_j - x_i < -L_a/2, -1 when > L_a/2) either merges two
 * clusters with the implied relative image, or closes a cycle, which winds
 * along the axes where the images disagree.  *mask = OR of those axes. */
static int64_t o_uf_find(int64_t *parent, int32_t (*off)[3], int64_t i, int32_t out[3])
{
    int32_t acc[3] = {0, 0, 0};
    int64_t r = i;
    while (parent[r] != r) {
        for (int a = 0; a < 3; ++a) acc[a] += off[r][a];
        r = parent[r];
    }
    /* path compression: point i (and its chain) at the root */
    int64_t k = i;
    int32_t rem[3] = {acc[0], acc[1], acc[2]};
    while (parent[k] != k) {
        int64_t next = parent[k];
        int32_t step[3] = {off[k][0], off[k][1], off[k][2]};
        parent[k] = r;
        for (int a = 0; a < 3; ++a) {
            off[k][a] = rem[a];
            rem[a] -= step[a];
        }
        k = next;
    }
    for (int a = 0; a < 3; ++a) out[a] = acc[a];
    return r;
}

int o_percolation(const o_state *st, double s, double gap, int32_t *mask)
{
    const o_params *p = &st->p;
    int64_t n = p->n;
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t (*off)[3] = (int32_t (*)[3])malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    if (!parent || !off) { free(parent); free(off); return O_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) {
        parent[i] = i;
        off[i][0] = off[i][1] = off[i][2] = 0;
    }
    *mask = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            int hit;
            if (p->shape == O_PLATELET) {
                double ai = o_radius(st, s, i) + 0.5 * gap, aj = o_radius(st, s, j) + 0.5 * gap;
                hit = o_disks_intersect(&st->pos[3 * i], &st->nrm[3 * i], ai,
                                        &st->pos[3 * j], &st->nrm[3 * j], aj, p->box);
            } else if (p->shape == O_SPHERODISK) {
                hit = o_spherodisks_overlap(&st->pos[3 * i], &st->nrm[3 * i], o_radius(st, s, i),
                                            &st->pos[3 * j], &st->nrm[3 * j], o_radius(st, s, j),
                                            p->thick_ratio, gap, p->box);
            } else {
                double sig = (o_radius(st, s, i) + o_radius(st, s, j)) + gap;
                hit = o_pair_q(st, i, j) <= sig * sig;
            }
            if (!hit) continue;
            int32_t sh[3] = {0, 0, 0};
            for (int a = 0; a < p->dim; ++a) {
                double d = st->pos[3 * j + a] - st->pos[3 * i + a];
                sh[a] = (d > 0.5 * p->box[a]) ? -1 : ((d < -0.5 * p->box[a]) ? 1 : 0);
            }
            /* image of i relative to its root oi, of j relative to its root oj;
             * the bond says image(j) = image(i) + sh */
            int32_t oi[3], oj[3];
            int64_t ri = o_uf_find(parent, off, i, oi);
            int64_t rj = o_uf_find(parent, off, j, oj);
            if (ri != rj) {
                parent[rj] = ri;
                for (int a = 0; a < 3; ++a) off[rj][a] = oi[a] + sh[a] - oj[a];
            } else {
                for (int a = 0; a < 3; ++a)
                    if (oi[a] + sh[a] != oj[a]) *mask |= 1 << a;
            }
        }
    }
    free(parent);
    free(off);
    return O_OK;
}

/* Histogram of centre distances r_ij (i<j): bin b = (int)(r * (nbins / r_max)),
 * counted when b < nbins. */
int o_rdf_brute(const o_state *st, int32_t nbins, double r_max, uint64_t *counts)
{
    double inv = (double)nbins / r_max;
    for (int32_t b = 0; b < nbins; ++b) counts[b] = 0;
    for (int64_t i = 0; i < st->p.n; ++i)
        for (int64_t j = i + 1; j < st->p.n; ++j) {
            double r = sqrt(o_pair_q(st, i, j));
            double x = r * inv;
            if (x < (double)nbins) {
                int64_t b = (int64_t)x;
                if (b < nbins) counts[b]++;
            }
        }
    return O_OK;
}

/* Nearest-neighbour distances (the structure descriptor of the paper's
 * Sec. 3.2 comparison, Fig. 4d): for every particle i the square root of the
 * smallest q_ij over all j != i with q_ij < r_max^2, or +infinity when
 * there is none.  All pairs. */
int o_nearest_brute(const o_state *st, double r_max, double *dist)
{
    double r2 = r_max * r_max;
    for (int64_t i = 0; i < st->p.n; ++i) {
        double best = r2;
        int found = 0;
        for (int64_t j = 0; j < st->p.n; ++j) {
            if (j == i) continue;
            double q = o_pair_q(st, i, j);
            if (q < best) {
                best = q;
                found = 1;
            }
        }
        dist[i] = found ? sqrt(best) : INFINITY;
    }
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Soft-binned radial distribution and overlap penalty (differentiable  */
/* steering of configurations toward a target g(r)).                   */
/*                                                                      */
/* Bins b = 0..nb-1 of width D = r_c / nb, centres c_b = (b + 1/2) D,   */
/* Gaussian kernel K_b(r) = exp(-(r - c_b)^2 / (2 h^2)) / (h sqrt(2 pi)) */
/* with h = D, and a C2 taper w(r) = 1 - 10t^3 + 15t^4 - 6t^5,          */
/* t = (r - r_c) / (4h) on [r_c, r_c + 4h] (1 before, 0 after).          */
/*   g_b = norm_b * sum_{i<j} K_b(r_ij) w(r_ij),                         */
/*   norm_b = V / (N(N-1)/2 * 4 pi c_b^2)   (3D; 2D: 2 pi c_b),          */
/*   E = kappa/2 * sum_{i<j} max(0, R_i + R_j - r_ij)^2,                 */
/* with r_ij the minimum-image distance.  All pairs, all in FP64.        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t dim, nbins;
    double box[3];
    double r_c;
    double kappa;
} o_softrdf_params;

static double o_taper(double r, double r_c, double h, double *dw)
{
    double span = 4.0 * h;
    if (r <= r_c) { *dw = 0.0; return 1.0; }
    if (r >= r_c + span) { *dw = 0.0; return 0.0; }
    double t = (r - r_c) / span;
    double t2 = t * t, t3 = t2 * t;
    *dw = (-30.0 * t2 + 60.0 * t3 - 30.0 * t2 * t2) / span;
    return 1.0 - 10.0 * t3 + 15.0 * t3 * t - 6.0 * t3 * t2;
}

static double o_soft_norm(const o_softrdf_params *p, int64_t n, int b)
{
    double D = p->r_c / p->nbins;
    double c = (b + 0.5) * D;
    double vol = 1.0;
    for (int a = 0; a < p->dim; ++a) vol *= p->box[a];
    double pairs = 0.5 * (double)n * (double)(n - 1);
    double shell = (p->dim == 3) ? 4.0 * M_PI * c * c : 2.0 * M_PI * c;
    return vol / (pairs * shell);
}

static void o_pair_vec(const o_softrdf_params *p, const double *xi, const double *xj, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        if (a >= p->dim) { d[a] = 0.0; continue; }
        d[a] = o_minimg(xi[a] - xj[a], p->box[a]);
    }
}

void o_softrdf_fwd(const o_softrdf_params *p, int64_t n, const double *pos, const double *radii,
                   double *g, double *energy)
{
    double D = p->r_c / p->nbins, h = D;
    double cut = p->r_c + 4.0 * h;
    double c0 = 1.0 / (h * sqrt(2.0 * M_PI));
    for (int b = 0; b < p->nbins; ++b) g[b] = 0.0;
    double E = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double d[3];
            o_pair_vec(p, &pos[3 * i], &pos[3 * j], d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double ov = radii[i] + radii[j] - r;
            if (ov > 0.0) E += ov * ov;
            if (r >= cut) continue;
            double dw;
            double w = o_taper(r, p->r_c, h, &dw);
            for (int b = 0; b < p->nbins; ++b) {
                double u = (r - (b + 0.5) * D) / h;
                g[b] += c0 * exp(-0.5 * u * u) * w;
            }
        }
    }
    for (int b = 0; b < p->nbins; ++b) g[b] *= o_soft_norm(p, n, b);
    *energy = 0.5 * p->kappa * E;
}

/* Gradient of L with dL/dg_b = dg[b] and dL/dE = dE with respect to every
 * position (n rows of 3) and radius. */
void o_softrdf_grad(const o_softrdf_params *p, int64_t n, const double *pos, const double *radii,
                    const double *dg, double dE, double *gpos, double *grad_r)
{
    double D = p->r_c / p->nbins, h = D;
    double cut = p->r_c + 4.0 * h;
    double c0 = 1.0 / (h * sqrt(2.0 * M_PI));
    for (int64_t i = 0; i < 3 * n; ++i) gpos[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) grad_r[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double d[3];
            o_pair_vec(p, &pos[3 * i], &pos[3 * j], d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r == 0.0) continue;
            /* dL/dr for this pair */
            double dLdr = 0.0;
            double ov = radii[i] + radii[j] - r;
            if (ov > 0.0) {
                dLdr += dE * p->kappa * (-ov);
                grad_r[i] += dE * p->kappa * ov;
                grad_r[j] += dE * p->kappa * ov;
            }
            if (r < cut) {
                double dw;
                double w = o_taper(r, p->r_c, h, &dw);
                for (int b = 0; b < p->nbins; ++b) {
                    double u = (r - (b + 0.5) * D) / h;
                    double k = c0 * exp(-0.5 * u * u);
                    double dk = k * (-u / h);
                    dLdr += dg[b] * o_soft_norm(p, n, b) * (dk * w + k * dw);
                }
            }
            for (int a = 0; a < p->dim; ++a) {
                double ua = d[a] / r;
                gpos[3 * i + a] += dLdr * ua;
                gpos[3 * j + a] -= dLdr * ua;
            }
        }
    }
}
