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

}  // namespace srm
