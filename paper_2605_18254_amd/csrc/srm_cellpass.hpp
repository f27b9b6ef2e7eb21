// srm_cellpass.hpp -- the per-cell migration pass and the per-particle
// overlap test on the global-memory layout, shared by the single-box kernels
// and the batched ensemble kernels.  A thread owns one cell of the current
// colour and runs Algorithm 3 for its particles in ascending id order; the
// collision test (Algorithm 5) scans the 3^dim stencil around the binned
// cell.  With a cell edge >= 2.5 R'max + 2.5 c_m every particle within
// R_i + R_j of a trial position lies in that stencil, so each decision
// equals the all-pairs test.
#pragma once

#include "srm_internal.hpp"

namespace srm {

// Does a ball of radius Ri at (yx, yy, yz) overlap any particle of the
// slices other than slot `self`?  q = (dx*dx + dy*dy) + dz*dz <= (Ri+Rj)^2.
template <int DIM, bool POLY, bool GENERAL>
__device__ __forceinline__ bool ball_hits(const PassArgs &a, const int32_t *lo, const int32_t *hi,
                                          int32_t self, double yx, double yy, double yz, double Ri)
{
    const double *__restrict__ X = a.buf.x[0];
    const double *__restrict__ Y = a.buf.x[1];
    const double *__restrict__ Z = a.buf.x[2];
#pragma unroll
    for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
        for (int32_t q = lo[r]; q < hi[r]; ++q) {
            if (q == self) continue;
            double dx = yx - X[q];
            double dy = yy - Y[q];
            if (GENERAL) {
                dx = min_image(dx, a.g.box[0], a.g.half[0]);
                dy = min_image(dy, a.g.box[1], a.g.half[1]);
            }
            double qq = dx * dx + dy * dy;
            if (DIM == 3) {
                double dz = yz - Z[q];
                if (GENERAL) dz = min_image(dz, a.g.box[2], a.g.half[2]);
                qq = qq + dz * dz;
            }
            double sig2;
            if (POLY) {
                const double sig = Ri + a.s * a.buf.rho[q];
                sig2 = sig * sig;
            } else {
                sig2 = a.sig2_mono;
            }
            if (qq <= sig2) return true;
        }
    }
    return false;
}

template <int DIM>
__device__ __forceinline__ bool is_interior(const Grid &g, int32_t cx, int32_t cy, int32_t cz)
{
    bool in = g.na[0] >= 8 && g.na[1] >= 8 && cx >= 2 && cx <= g.na[0] - 3 && cy >= 2 &&
              cy <= g.na[1] - 3;
    if (DIM == 3) in = in && g.na[2] >= 8 && cz >= 2 && cz <= g.na[2] - 3;
    return in;
}

// Algorithm 3 for the particles of one cell (global-memory path): slots
// [beg, end) in ascending id order, each with up to N_l trials.
template <int DIM, bool POLY>
__device__ __forceinline__ void migrate_cell_global(const PassArgs &a, int32_t cx, int32_t cy,
                                                    int32_t cz)
{
    const int32_t c = cx + a.g.na[0] * (cy + a.g.na[1] * cz);
    const int32_t beg = a.start[c], end = a.start[c + 1];
    if (beg == end) return;
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
    const bool general = !is_interior<DIM>(a.g, cx, cy, cz);
    double *__restrict__ X = a.buf.x[0];
    double *__restrict__ Y = a.buf.x[1];
    double *__restrict__ Z = a.buf.x[2];
    for (int32_t p = beg; p < end; ++p) {
        const double ox = X[p], oy = Y[p], oz = (DIM == 3) ? Z[p] : 0.0;
        const uint32_t id = (uint32_t)a.buf.id[p];
        const double Ri = POLY ? a.s * a.buf.rho[p] : a.s;
        uint8_t code = 0;
        Draw d = a.draw;
        for (int32_t l = 1; l <= a.n_l; ++l) {
            double v[3];
            d.word = a.draw.word | ((uint32_t)l << 8);
            unit_vector<DIM>(d, id, 0, a.c_m, v);
            const double yx = wrap_coord(ox + v[0], a.g.box[0]);
            const double yy = wrap_coord(oy + v[1], a.g.box[1]);
            const double yz = (DIM == 3) ? wrap_coord(oz + v[2], a.g.box[2]) : 0.0;
            const bool hit = general ? ball_hits<DIM, POLY, true>(a, lo, hi, p, yx, yy, yz, Ri)
                                     : ball_hits<DIM, POLY, false>(a, lo, hi, p, yx, yy, yz, Ri);
            if (!hit) {
                X[p] = yx;
                Y[p] = yy;
                if (DIM == 3) Z[p] = yz;
                code = (uint8_t)l;
                break;
            }
        }
        a.acc[p] = code;
        if (code == 0) a.failed[1 + atomicAdd(&a.failed[0], 1)] = p;
    }
}

// Algorithm 6 for the particle in slot p at its current position.
template <int DIM, bool POLY>
__device__ __forceinline__ bool check_ball_one(const PassArgs &a, int32_t p)
{
    const double x = a.buf.x[0][p], y = a.buf.x[1][p];
    const double z = (DIM == 3) ? a.buf.x[2][p] : 0.0;
    const int32_t cx = cell_coord(x, a.g.inv_w[0], a.g.na[0]);
    const int32_t cy = cell_coord(y, a.g.inv_w[1], a.g.na[1]);
    const int32_t cz = (DIM == 3) ? cell_coord(z, a.g.inv_w[2], a.g.na[2]) : 0;
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
    const double Ri = POLY ? a.s * a.buf.rho[p] : a.s;
    return ball_hits<DIM, POLY, true>(a, lo, hi, p, x, y, z, Ri);
}

// Algorithm 6 for the particle in slot p, its stencil split over the 64
// lanes of a wavefront (crowded cells hold tens of particles, so one lane's
// scan would be a long chain of dependent loads): the same exact test as
// check_ball_one, any lane's hit counts.
template <int DIM, bool POLY>
__device__ __forceinline__ bool check_ball_wave(const PassArgs &a, int32_t p, int lane)
{
    const double *__restrict__ X = a.buf.x[0];
    const double *__restrict__ Y = a.buf.x[1];
    const double *__restrict__ Z = a.buf.x[2];
    const double x = X[p], y = Y[p];
    const double z = (DIM == 3) ? Z[p] : 0.0;
    const int32_t cx = cell_coord(x, a.g.inv_w[0], a.g.na[0]);
    const int32_t cy = cell_coord(y, a.g.inv_w[1], a.g.na[1]);
    const int32_t cz = (DIM == 3) ? cell_coord(z, a.g.inv_w[2], a.g.na[2]) : 0;
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
    const double Ri = POLY ? a.s * a.buf.rho[p] : a.s;
    bool hit = false;
#pragma unroll
    for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
        for (int32_t q = lo[r] + lane; q < hi[r] && !hit; q += 64) {
            if (q == p) continue;
            const double dx = min_image(x - X[q], a.g.box[0], a.g.half[0]);
            const double dy = min_image(y - Y[q], a.g.box[1], a.g.half[1]);
            double qq = dx * dx + dy * dy;
            if (DIM == 3) {
                const double dz = min_image(z - Z[q], a.g.box[2], a.g.half[2]);
                qq = qq + dz * dz;
            }
            double sig2;
            if (POLY) {
                const double sig = Ri + a.s * a.buf.rho[q];
                sig2 = sig * sig;
            } else {
                sig2 = a.sig2_mono;
            }
            hit = qq <= sig2;
        }
    }
    return __ballot(hit) != 0;
}

// ---- one wavefront per cell ------------------------------------------------
//
// For crowded cells (polydisperse boxes put tens of particles in a cell,
// whose edge follows the largest radius) the whole 64-lane wavefront of a
// 64-thread workgroup runs Algorithm 3 for one cell:
//  A. the cell's particles go to LDS and each gets a near list: stencil
//     candidates outside the cell within R_i + R_j + 2 c_m of it (they do
//     not move in this colour phase, and a trial lies within c_m of the old
//     position), and the cell's other particles within R_i + R_j + 3 c_m
//     (each moves at most c_m before i's turn; the extra c_m is slack for
//     rounding).  Lanes split the candidates.
//  B. first, in parallel, each particle's first trial that misses its
//     near-list candidates outside the cell (fixed during the phase); then
//     particles in ascending id order: that trial wins if it also misses
//     the cell mates at their current LDS positions, else the lanes split
//     (trial, near entry) pairs of a group of the following trials and the
//     lowest collision-free trial of the group wins -- the first free trial
//     of the sequential rule, since no trial of one particle changes what
//     another trial of it sees.
// A particle whose near list overflows tests its trials one at a time
// against the whole stencil; a cell with more than kWaveOwn particles runs
// on one lane with the global-memory routine above.
constexpr int kWaveOwn = 96;
constexpr int kWaveNear = 24;
constexpr int kWaveOccupancy = 3;  // mean particles per cell that selects this path

struct WaveOwn {
    double x, y, z, r;
};

struct WaveLds {
    WaveOwn own[kWaveOwn];
    float4 own32[kWaveOwn];  // own particles rounded to FP32, for the near-list filter
    int32_t nn[kWaveOwn];
    int32_t near[kWaveOwn * kWaveNear];  // slot q >= 0, or -(k + 1) for own particle k
    int32_t id[kWaveOwn];
    int32_t nfail;
    union {
        int32_t fail[kWaveOwn];  // phase B: own indices that rejected every trial
        int32_t kept[128];       // phase A: stencil candidates near the cell, queued
    };
};

template <int DIM>
__device__ __forceinline__ double wave_q(const Grid &g, double ax, double ay, double az, double bx,
                                         double by, double bz)
{
    const double dx = min_image(ax - bx, g.box[0], g.half[0]);
    const double dy = min_image(ay - by, g.box[1], g.half[1]);
    double qq = dx * dx + dy * dy;
    if (DIM == 3) {
        const double dz = min_image(az - bz, g.box[2], g.half[2]);
        qq = qq + dz * dz;
    }
    return qq;
}

// Trial l of the particle with id `id` at (ox, oy, oz): Algorithm 3's
// wrapped position.
template <int DIM>
__device__ __forceinline__ void wave_trial(const PassArgs &a, uint32_t id, int32_t l, double ox,
                                           double oy, double oz, double &yx, double &yy,
                                           double &yz)
{
    Draw d = a.draw;
    d.word = a.draw.word | ((uint32_t)l << 8);
    double v[3];
    unit_vector<DIM>(d, id, 0, a.c_m, v);
    yx = wrap_coord(ox + v[0], a.g.box[0]);
    yy = wrap_coord(oy + v[1], a.g.box[1]);
    yz = (DIM == 3) ? wrap_coord(oz + v[2], a.g.box[2]) : 0.0;
}

// Exact Algorithm 5 predicate of a trial (radius Ri) against one candidate,
// evaluated as in ball_hits: q = (dx*dx + dy*dy) + dz*dz <= (Ri + Rc)^2.
template <int DIM, bool POLY>
__device__ __forceinline__ bool wave_hit(const PassArgs &a, double yx, double yy, double yz,
                                         double Ri, double cx, double cy, double cz, double Rc)
{
    const double dx = min_image(yx - cx, a.g.box[0], a.g.half[0]);
    const double dy = min_image(yy - cy, a.g.box[1], a.g.half[1]);
    double qq = dx * dx + dy * dy;
    if (DIM == 3) {
        const double dz = min_image(yz - cz, a.g.box[2], a.g.half[2]);
        qq = qq + dz * dz;
    }
    double sig2;
    if (POLY) {
        const double sig = Ri + Rc;
        sig2 = sig * sig;
    } else {
        sig2 = a.sig2_mono;
    }
    return qq <= sig2;
}

// Near-list entry `ref` against a trial of own particle k.
template <int DIM, bool POLY>
__device__ __forceinline__ bool wave_ref_hit(const PassArgs &a, const WaveLds &L, int32_t ref,
                                             double yx, double yy, double yz, double Ri)
{
    if (ref < 0) {
        const WaveOwn o = L.own[-ref - 1];
        return wave_hit<DIM, POLY>(a, yx, yy, yz, Ri, o.x, o.y, o.z, o.r);
    }
    return wave_hit<DIM, POLY>(a, yx, yy, yz, Ri, a.buf.x[0][ref], a.buf.x[1][ref],
                               (DIM == 3) ? a.buf.x[2][ref] : 0.0,
                               POLY ? a.s * a.buf.rho[ref] : a.s);
}

// Algorithm 3 for the particles of one cell, G consecutive lanes of a
// wavefront per cell (G divides 64; the G lanes call it uniformly).  The
// particles are still taken one at a time in ascending id order and each
// one's trials in order; the lanes split a trial's stencil (every G-th
// candidate of each slice), and the trial is accepted when none of them
// finds a contact (Algorithm 5, the test of ball_hits).  Every lane of the
// group stores the accepted position, so each lane's later reads of that
// slot follow its own store.
template <int DIM, bool POLY, int G>
__device__ __forceinline__ void migrate_cell_lanes(const PassArgs &a, int32_t cx, int32_t cy,
                                                   int32_t cz)
{
    static_assert(64 % G == 0, "a group stays inside one wavefront");
    const int lane = threadIdx.x & 63;
    const int32_t sub = lane % G;
    const int32_t c = cx + a.g.na[0] * (cy + a.g.na[1] * cz);
    const int32_t beg = a.start[c], end = a.start[c + 1];
    if (beg == end) return;  // group-uniform
    int32_t slo[Rows<DIM>::kRanges], shi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, slo, shi);
    constexpr unsigned long long kOnes = (G == 64) ? ~0ull : ((1ull << (G % 64)) - 1);
    const unsigned long long gmask = kOnes << (lane & ~(G - 1));
    double *__restrict__ X = a.buf.x[0];
    double *__restrict__ Y = a.buf.x[1];
    double *__restrict__ Z = a.buf.x[2];
    for (int32_t p = beg; p < end; ++p) {
        const double ox = X[p], oy = Y[p], oz = (DIM == 3) ? Z[p] : 0.0;
        const uint32_t id = (uint32_t)a.buf.id[p];
        const double Ri = POLY ? a.s * a.buf.rho[p] : a.s;
        int32_t code = 0;
        for (int32_t l = 1; l <= a.n_l; ++l) {
            double yx, yy, yz;
            wave_trial<DIM>(a, id, l, ox, oy, oz, yx, yy, yz);
            bool hit = false;
#pragma unroll 1  // unrolled, each slice's loop is pipelined apart (255 VGPRs)
            for (int k = 0; k < Rows<DIM>::kRanges; ++k) {
                for (int32_t q = slo[k] + sub; q < shi[k] && !hit; q += G) {
                    if (q == p) continue;
                    hit = wave_hit<DIM, POLY>(a, yx, yy, yz, Ri, X[q], Y[q],
                                              (DIM == 3) ? Z[q] : 0.0,
                                              POLY ? a.s * a.buf.rho[q] : a.s);
                }
            }
            if ((__ballot(hit) & gmask) == 0) {
                X[p] = yx;
                Y[p] = yy;
                if (DIM == 3) Z[p] = yz;
                code = l;
                break;
            }
        }
        if (sub == 0) {
            a.acc[p] = (uint8_t)code;
            if (code == 0) a.failed[1 + atomicAdd(&a.failed[0], 1)] = p;
        }
    }
}

// Must be called by all 64 threads of a 64-thread workgroup, uniformly.
template <int DIM, bool POLY>
__device__ void migrate_cell_wave(const PassArgs &a, int32_t cx, int32_t cy, int32_t cz,
                                  WaveLds &L)
{
    const int lane = threadIdx.x;
    const int32_t c = cx + a.g.na[0] * (cy + a.g.na[1] * cz);
    const int32_t beg = a.start[c], end = a.start[c + 1];
    const int32_t cnt = end - beg;
    if (cnt == 0) return;
    if (cnt > kWaveOwn) {  // beyond LDS: the stencil split over the lanes
        migrate_cell_lanes<DIM, POLY, 64>(a, cx, cy, cz);
        return;
    }
    const double *__restrict__ X = a.buf.x[0];
    const double *__restrict__ Y = a.buf.x[1];
    const double *__restrict__ Z = a.buf.x[2];
    int32_t lo[Rows<DIM>::kRanges], hi[Rows<DIM>::kRanges];
    stencil_slices<DIM>(a.g, a.start, cx, cy, cz, lo, hi);
    float rmax32 = 0.0f;  // largest own radius, for the cell-box filter below
    for (int32_t k = lane; k < cnt; k += 64) {
        WaveOwn o;
        o.x = X[beg + k];
        o.y = Y[beg + k];
        o.z = (DIM == 3) ? Z[beg + k] : 0.0;
        o.r = POLY ? a.s * a.buf.rho[beg + k] : a.s;
        L.own[k] = o;
        L.own32[k] = make_float4((float)o.x, (float)o.y, (float)o.z, (float)o.r);
        rmax32 = fmaxf(rmax32, (float)o.r);
        L.nn[k] = 0;
        L.id[k] = a.buf.id[beg + k];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rmax32 = fmaxf(rmax32, __shfl_xor(rmax32, o, 64));
    if (lane == 0) L.nfail = 0;
    __syncthreads();
    // A. near lists.  A list only has to contain every candidate that can
    // meet a trial (the exact FP64 test decides later), so the filter runs
    // in FP32 with a margin that covers rounding: positions in [0, L) are
    // off by at most L 2^-24 each, so each difference by ~3 L 2^-24 after the
    // image shift; 4e-7 Lmax absolute plus 1e-5 relative on the reach bounds
    // that with room to spare.  Extra entries only cost time.
    const float bx32 = (float)a.g.box[0], by32 = (float)a.g.box[1], bz32 = (float)a.g.box[2];
    const float hx32 = 0.5f * bx32, hy32 = 0.5f * by32, hz32 = 0.5f * bz32;
    float lmax32 = bx32 > by32 ? bx32 : by32;
    if (DIM == 3) lmax32 = lmax32 > bz32 ? lmax32 : bz32;
    const float tol32 = 4e-7f * lmax32;
    auto near32 = [&](const float4 &o, float px, float py, float pz, float reach) {
        float dx = o.x - px, dy = o.y - py;
        if (dx > hx32) dx -= bx32;
        if (dx < -hx32) dx += bx32;
        if (dy > hy32) dy -= by32;
        if (dy < -hy32) dy += by32;
        float qq = dx * dx + dy * dy;
        if (DIM == 3) {
            float dz = o.z - pz;
            if (dz > hz32) dz -= bz32;
            if (dz < -hz32) dz += bz32;
            qq = qq + dz * dz;
        }
        const float rr = reach * 1.00001f + tol32;
        return qq <= rr * rr;
    };
    const float cm2 = (float)(2.0 * a.c_m), cm3 = (float)(3.0 * a.c_m);
    // Every own particle sits in the cell's box (binned this pass, not yet
    // moved), so a candidate farther from the box than R_q + max R_own +
    // 2 c_m meets none of them.  The box test keeps a superset of what the
    // pair filter keeps (three times its rounding margin), and with a cell
    // edge set by the largest radius it drops most of the stencil.  Kept
    // candidates queue in LDS and are tested against the own particles 64 at
    // a time, so the lanes of a pass all carry one.
    const double wxd = a.g.box[0] / (double)a.g.na[0], wyd = a.g.box[1] / (double)a.g.na[1];
    const double wzd = (DIM == 3) ? a.g.box[2] / (double)a.g.na[2] : 0.0;
    const float ccx = (float)((cx + 0.5) * wxd), ccy = (float)((cy + 0.5) * wyd);
    const float ccz = (float)((cz + 0.5) * wzd);
    const float hwx = (float)(0.5 * wxd), hwy = (float)(0.5 * wyd), hwz = (float)(0.5 * wzd);
    auto box_gap = [](float d, float h, float b, float hw) {
        if (d > h) d -= b;
        if (d < -h) d += b;
        const float g = fabsf(d) - hw;
        return g > 0.0f ? g : 0.0f;
    };
    // With at least four cells on every axis the cell edge is at most L/4
    // and at least the largest reach, so a candidate within reach of an own
    // particle lies within 1.5 edges of the cell's centre.  Shifted once to
    // the image nearest that centre, its difference to every own particle
    // is then the minimum image whenever it is within reach (and never
    // smaller otherwise), as is the difference of two own particles: the
    // pair filters need no per-pair wrap.  The shift adds one rounding of
    // at most L 2^-24, inside the margin above.
    const bool direct = a.g.na[0] >= 4 && a.g.na[1] >= 4 && (DIM == 2 || a.g.na[2] >= 4);
    auto near32d = [&](const float4 &o, float px, float py, float pz, float reach) {
        const float dx = o.x - px, dy = o.y - py;
        float qq = dx * dx + dy * dy;
        if (DIM == 3) {
            const float dz = o.z - pz;
            qq = qq + dz * dz;
        }
        const float rr = reach * 1.00001f + tol32;
        return qq <= rr * rr;
    };
    auto to_centre = [](float q, float c, float h, float b) {
        const float d = q - c;
        return d > h ? q - b : (d < -h ? q + b : q);
    };
    auto pair_pass = [&](int32_t q) {
        float qx = (float)X[q], qy = (float)Y[q], qz = (DIM == 3) ? (float)Z[q] : 0.0f;
        const float Rq = (float)(POLY ? a.s * a.buf.rho[q] : a.s);
        if (direct) {
            qx = to_centre(qx, ccx, hx32, bx32);
            qy = to_centre(qy, ccy, hy32, by32);
            if (DIM == 3) qz = to_centre(qz, ccz, hz32, bz32);
#pragma unroll 4  // independent list appends of four own particles overlap
            for (int32_t k = 0; k < cnt; ++k) {
                const float4 o = L.own32[k];
                if (near32d(o, qx, qy, qz, (o.w + Rq) + cm2)) {
                    const int32_t slot = atomicAdd(&L.nn[k], 1);
                    if (slot < kWaveNear) L.near[k * kWaveNear + slot] = q;
                }
            }
            return;
        }
#pragma unroll 4
        for (int32_t k = 0; k < cnt; ++k) {
            const float4 o = L.own32[k];
            if (near32(o, qx, qy, qz, (o.w + Rq) + cm2)) {
                const int32_t slot = atomicAdd(&L.nn[k], 1);
                if (slot < kWaveNear) L.near[k * kWaveNear + slot] = q;
            }
        }
    };
    int32_t nk = 0;  // queued candidates (the same in every lane)
#pragma unroll
    for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
        for (int32_t q0 = lo[r]; q0 < hi[r]; q0 += 64) {
            const int32_t q = q0 + lane;
            bool keep = false;
            if (q < hi[r] && !(q >= beg && q < end)) {
                const float qx = (float)X[q], qy = (float)Y[q];
                const float qz = (DIM == 3) ? (float)Z[q] : 0.0f;
                const float Rq = (float)(POLY ? a.s * a.buf.rho[q] : a.s);
                const float gx = box_gap(qx - ccx, hx32, bx32, hwx);
                const float gy = box_gap(qy - ccy, hy32, by32, hwy);
                float g2 = gx * gx + gy * gy;
                if (DIM == 3) {
                    const float gz = box_gap(qz - ccz, hz32, bz32, hwz);
                    g2 = g2 + gz * gz;
                }
                const float rr = ((Rq + rmax32) + cm2) * 1.00001f + 3.0f * tol32;
                keep = g2 <= rr * rr;
            }
            const unsigned long long km = __ballot(keep);
            if (keep) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
                L.kept[nk + (int32_t)below] = q;
            }
            nk += __popcll(km);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (nk >= 64) {
                pair_pass(L.kept[lane]);
                const int32_t rem = nk - 64;
                const int32_t mv = (lane < rem) ? L.kept[64 + lane] : 0;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane < rem) L.kept[lane] = mv;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                nk = rem;
            }
        }
    }
    if (lane < nk) pair_pass(L.kept[lane]);
    for (int32_t j = lane; j < cnt; j += 64) {
        const float4 b = L.own32[j];
#pragma unroll 4  // independent list appends of four own particles overlap
        for (int32_t k = 0; k < cnt; ++k) {
            if (k == j) continue;
            const float4 o = L.own32[k];
            if (direct ? near32d(o, b.x, b.y, b.z, (o.w + b.w) + cm3)
                       : near32(o, b.x, b.y, b.z, (o.w + b.w) + cm3)) {
                const int32_t slot = atomicAdd(&L.nn[k], 1);
                if (slot < kWaveNear) L.near[k * kWaveNear + slot] = -(j + 1);
            }
        }
    }
    __syncthreads();
    // B. the sequential part.  Cell mates are read from LDS at test time;
    // near-list candidates outside the cell (fixed in this phase) are read
    // from global memory only by the trials after a speculated one failed.
    // B0. Lane j takes own particles j and j + 64 and finds each one's first
    // trial that meets no near-list candidate outside the cell: those
    // candidates do not move in this phase, so the trials before it are
    // rejected whatever the cell mates do (-1: near list overflowed, not
    // looked at; 0: every trial meets one).
    int32_t spec[2] = {-1, -1};
    double sxv[2] = {0.0, 0.0}, syv[2] = {0.0, 0.0}, szv[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t k = lane + 64 * h;
        if (k >= cnt || L.nn[k] > kWaveNear) continue;
        const int32_t m = L.nn[k];
        const WaveOwn me = L.own[k];
        const uint32_t id = (uint32_t)L.id[k];
        spec[h] = 0;
        for (int32_t l = 1; l <= a.n_l; ++l) {
            double yx, yy, yz;
            wave_trial<DIM>(a, id, l, me.x, me.y, me.z, yx, yy, yz);
            // near entries four at a time: their loads are issued together
            bool hit = false;
            for (int32_t e = 0; e < m && !hit; e += 4) {
                int32_t rf[4];
                double qx[4], qy[4], qz[4], qr[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    rf[i] = (e + i < m) ? L.near[k * kWaveNear + e + i] : -1;
                    qx[i] = qy[i] = qz[i] = qr[i] = 0.0;
                    if (rf[i] >= 0) {
                        qx[i] = X[rf[i]];
                        qy[i] = Y[rf[i]];
                        if (DIM == 3) qz[i] = Z[rf[i]];
                        qr[i] = POLY ? a.s * a.buf.rho[rf[i]] : a.s;
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (rf[i] >= 0)
                        hit = hit || wave_hit<DIM, POLY>(a, yx, yy, yz, me.r, qx[i], qy[i], qz[i],
                                                         qr[i]);
            }
            if (!hit) {
                spec[h] = l;
                sxv[h] = yx;
                syv[h] = yy;
                szv[h] = yz;
                break;
            }
        }
    }
    for (int32_t k = 0; k < cnt; ++k) {
        const int32_t p = beg + k;
        const WaveOwn me = L.own[k];
        const uint32_t id = (uint32_t)L.id[k];
        const int32_t m = L.nn[k];
        int32_t code = 0;
        double wx = 0.0, wy = 0.0, wz = 0.0;
        // B1. settle the speculated trial against the cell mates at their
        // current positions; on a hit the remaining trials follow below
        const int h = k >> 6, src = k & 63;
        const int32_t l1 = __shfl(h ? spec[1] : spec[0], src, 64);
        int32_t first = 1;
        bool done = false;
        if (l1 == 0) {
            done = true;
        } else if (l1 > 0) {
            const double tx = __shfl(h ? sxv[1] : sxv[0], src, 64);
            const double ty = __shfl(h ? syv[1] : syv[0], src, 64);
            const double tz = __shfl(h ? szv[1] : szv[0], src, 64);
            bool hit = false;
            for (int32_t j = lane; j < cnt; j += 64) {
                if (j == k) continue;
                const WaveOwn o = L.own[j];
                hit = hit || wave_hit<DIM, POLY>(a, tx, ty, tz, me.r, o.x, o.y, o.z, o.r);
            }
            if (__ballot(hit) == 0) {
                done = true;
                code = l1;
                wx = tx;
                wy = ty;
                wz = tz;
            } else {
                first = l1 + 1;
            }
        }
        if (done) {
        } else if (m == 0) {
            // nothing within reach: the first trial is free
            wave_trial<DIM>(a, id, 1, me.x, me.y, me.z, wx, wy, wz);
            code = (a.n_l >= 1) ? 1 : 0;
        } else if (m <= kWaveNear) {
            const int32_t G = 64 / m;
            const int32_t g = lane / m, j = lane - g * m;
            const unsigned long long seg = (m == 64) ? ~0ull : ((1ull << m) - 1ull);
            const int32_t ref = L.near[k * kWaveNear + j];
            double qx = 0.0, qy = 0.0, qz = 0.0, qr = 0.0;
            if (g < G && ref >= 0) {
                qx = X[ref];
                qy = Y[ref];
                qz = (DIM == 3) ? Z[ref] : 0.0;
                qr = POLY ? a.s * a.buf.rho[ref] : a.s;
            }
            for (int32_t l0 = first; l0 <= a.n_l && code == 0; l0 += G) {
                const int32_t l = l0 + g;
                const bool active = g < G && l <= a.n_l;
                double yx, yy, yz;
                wave_trial<DIM>(a, id, active ? l : l0, me.x, me.y, me.z, yx, yy, yz);
                bool hit = false;
                if (active) {
                    if (ref < 0) {
                        const WaveOwn o = L.own[-ref - 1];
                        hit = wave_hit<DIM, POLY>(a, yx, yy, yz, me.r, o.x, o.y, o.z, o.r);
                    } else {
                        hit = wave_hit<DIM, POLY>(a, yx, yy, yz, me.r, qx, qy, qz, qr);
                    }
                }
                const unsigned long long hits = __ballot(hit);
                int32_t win = -1;
                for (int32_t gg = 0; gg < G && l0 + gg <= a.n_l; ++gg) {
                    if (((hits >> (gg * m)) & seg) == 0) {
                        win = gg;
                        break;
                    }
                }
                if (win >= 0) {
                    code = l0 + win;
                    wx = __shfl(yx, win * m, 64);
                    wy = __shfl(yy, win * m, 64);
                    wz = __shfl(yz, win * m, 64);
                }
            }
        } else {
            // near list overflowed: the whole stencil, one trial at a time
            for (int32_t l = first; l <= a.n_l && code == 0; ++l) {
                double yx, yy, yz;
                wave_trial<DIM>(a, id, l, me.x, me.y, me.z, yx, yy, yz);
                bool hit = false;
#pragma unroll
                for (int r = 0; r < Rows<DIM>::kRanges; ++r) {
                    for (int32_t q = lo[r] + lane; q < hi[r]; q += 64) {
                        if (q >= beg && q < end) continue;
                        hit = hit || wave_ref_hit<DIM, POLY>(a, L, q, yx, yy, yz, me.r);
                    }
                }
                for (int32_t j = lane; j < cnt; j += 64)
                    if (j != k) hit = hit || wave_ref_hit<DIM, POLY>(a, L, -(j + 1), yx, yy, yz, me.r);
                if (__ballot(hit) == 0) {
                    code = l;
                    wx = yx;
                    wy = yy;
                    wz = yz;
                }
            }
        }
        if (lane == 0) {
            if (code) {
                L.own[k].x = wx;
                L.own[k].y = wy;
                L.own[k].z = wz;
                a.buf.x[0][p] = wx;
                a.buf.x[1][p] = wy;
                if (DIM == 3) a.buf.x[2][p] = wz;
            } else {
                L.fail[L.nfail++] = k;
            }
            a.acc[p] = (uint8_t)code;
        }
        // The workgroup is this one wavefront, whose LDS operations complete
        // in order: lane 0's stores only need to be ordered before the next
        // particle's loads (a workgroup barrier here would also wait for the
        // global stores on every particle).
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the cell's failures go to the global list once, off the chain
    const int32_t nf = L.nfail;
    if (nf > 0) {
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&a.failed[0], nf);
        base = __shfl(base, 0, 64);
        for (int32_t i = lane; i < nf; i += 64) a.failed[1 + base + i] = beg + L.fail[i];
    }
}

}  // namespace srm
