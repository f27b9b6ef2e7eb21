// k_migrate.hip -- Algorithm 3 (move particles) with Algorithm 5 (collision
// check) over the 2^dim-colour cell schedule, and the global check of
// Algorithm 6.
//
// Schedule: one launch per colour g; a thread owns one cell whose parity
// vector is g and processes that cell's particles in ascending id order,
// each with up to N_l trial moves.  Cells of one colour are at least two
// cells apart on some axis, so no thread reads a cell another thread of the
// same launch writes, and the launch equals any sequential order of its
// cells.  The stencil is taken around the particle's binned cell; with a cell
// edge >= 2.5 R'max + 2.5 c_m every particle within R_i + R_j of a trial
// position is inside it, so each accept/reject decision equals the
// all-pairs test.
//
// Interior cells (2 <= c_a <= N_a - 3 on every axis, all N_a >= 8) cannot
// see a periodic image: neither the trial position nor any candidate has
// wrapped, and all differences are below L/2, so the minimum-image
// correction is the identity there and is skipped.
#include <math.h>

#include "srm_cellpass.hpp"

namespace srm {

namespace {

constexpr int kBlock = 256;


// One 64-thread workgroup per colour cell (crowded cells).
template <int DIM, bool POLY>
__global__ void __launch_bounds__(64) k_migrate_wave(PassArgs a, ColourLattice L)
{
    __shared__ WaveLds lds;
    const int32_t t = blockIdx.x;
    const int32_t jx = t % L.h[0];
    const int32_t r1 = t / L.h[0];
    const int32_t jy = r1 % L.h[1];
    const int32_t jz = r1 / L.h[1];
    migrate_cell_wave<DIM, POLY>(a, 2 * jx + L.off[0], 2 * jy + L.off[1],
                                 (DIM == 3) ? 2 * jz + L.off[2] : 0, lds);
}

// ------------------------------------------------------------ tiled kernel
//
// A 256-thread workgroup owns a tile of 64 cells of the launch's colour
// (4x4x4 in 3D, 8x8 in 2D) and stages the (2T+1)^dim cells around them --
// every cell its lanes can touch -- into LDS as SoA positions with a local
// CSR index; each thread copies whole cells so neighbouring threads read
// neighbouring addresses.  Then, with four lanes (a quad) per task:
//  A. near lists, in parallel over all particles of the tile's own cells,
//     one lane per (particle, stencil row): the candidates of the 3^dim
//     stencil outside the particle's own cell whose distance to its old
//     position is at most R_i + R_j + 2 c_m.  No such candidate moves
//     during this colour phase, and every particle a trial within c_m of the
//     old position can touch is among them (the exact test decides).
//  B. the sequential part, one quad per cell, particles in ascending id
//     order.  Each particle's first trial free of its near list is found
//     beforehand (lane per particle for trial 1, the whole quad four trials
//     at a time for the rest) and settled against the cell mates; failing
//     that, lane j of the quad draws trial l = base + j and tests it exactly
//     against the near list and the other particles of its own cell at their
//     current positions; the lowest collision-free trial of the batch is
//     accepted -- the first free trial of the sequential rule, since all
//     trials of one particle see the same neighbour state.
// Accepted moves go to LDS (later particles of the cell see them) and HBM.
// No quad reads a cell another quad writes (same colour), so LDS needs no
// synchronisation in phase B.  A tile whose neighbourhood does not fit LDS
// is queued for the global-memory kernel.

template <int DIM, bool POLY, int V = 0>  // V: LDS region class 0 standard, 1 mid, 2 wide
struct QuadCfg {
    static constexpr int T = (DIM == 3) ? 4 : 8;
    static constexpr int R = 2 * T + 1;
    static constexpr int kCells = (DIM == 3) ? R * R * R : R * R;
    static constexpr int kThreads = 256;
    static constexpr int kPer = (kCells + kThreads - 1) / kThreads;
    static constexpr int kNear = 11;    // near-list entries per particle
    // particles of the tile's own cells
    static constexpr int kOwn = (V == 2) ? 256 : (V == 1) ? 224 : 160;
    // LDS capacity in particles: the workgroup stays under 40 KB so four
    // workgroups (sixteen waves) fit a CU; the wide variant for denser grids
    // stays under 60 KB (two workgroups a CU).
    static constexpr int kCap = (DIM == 3) ? (POLY ? ((V == 2) ? 1632 : (V == 1) ? 1320 : 1080)
                                                   : ((V == 2) ? 2176 : (V == 1) ? 1744 : 1456))
                                           : (POLY ? 1464 : 2168);
};

struct TileLattice {
    int32_t h[3];      // colour cells per axis
    int32_t off[3];    // parity offset per axis
    int32_t nt[3];     // tiles per axis
    int32_t tiles;     // total tiles
    int32_t per_xcd;   // tiles per XCD chunk (ceil(tiles / 8))
    int32_t colour;
    int32_t *ovf;      // [8] counts, then 8 lists of max_tiles tile ids
    int32_t max_tiles;
};

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

// Bits of the calling lane's quad in a wave-wide ballot.
__device__ __forceinline__ uint32_t quad_bits(unsigned long long m)
{
    const int sh = (threadIdx.x & 63) & ~3;
    return (uint32_t)(m >> sh) & 0xFu;
}

template <int DIM>
__device__ __forceinline__ void tile_coords(const TileLattice &L, int32_t tile, int32_t &tx,
                                            int32_t &ty, int32_t &tz)
{
    tx = tile % L.nt[0];
    ty = (tile / L.nt[0]) % L.nt[1];
    tz = (DIM == 3) ? tile / (L.nt[0] * L.nt[1]) : 0;
}

// Squared distance (d0*d0 + d1*d1) + d2*d2 of two points, with the
// minimum-image correction when GENERAL.
template <int DIM, bool GENERAL>
__device__ __forceinline__ double sq_dist(const Grid &g, double ax, double ay, double az,
                                          double bx, double by, double bz)
{
    double dx = ax - bx, dy = ay - by;
    if (GENERAL) {
        dx = min_image(dx, g.box[0], g.half[0]);
        dy = min_image(dy, g.box[1], g.half[1]);
    }
    double qq = dx * dx + dy * dy;
    if (DIM == 3) {
        double dz = az - bz;
        if (GENERAL) dz = min_image(dz, g.box[2], g.half[2]);
        qq = qq + dz * dz;
    }
    return qq;
}

// Exact contact test of a ball of radius Ri at y against every particle of
// the 3^dim stencil of region cell (rx, ry, rz) except LDS slot `self`.
template <int DIM, bool POLY, bool GENERAL>
__device__ __forceinline__ bool lds_hits(const PassArgs &a, const double *sx, const double *sy,
                                         const double *sz, const double *srho,
                                         const uint16_t *lst, int32_t rx, int32_t ry, int32_t rz,
                                         int32_t self, double yx, double yy, double yz, double Ri)
{
    using C = QuadCfg<DIM, POLY>;
#pragma unroll
    for (int iz = 0; iz < (DIM == 3 ? 3 : 1); ++iz) {
#pragma unroll
        for (int iy = 0; iy < 3; ++iy) {
            const int32_t row = (ry + iy - 1) * C::R + ((DIM == 3) ? (rz + iz - 1) * C::R * C::R : 0);
            const int32_t lo = lst[row + rx - 1], hi = lst[row + rx + 2];
            for (int32_t q = lo; q < hi; ++q) {
                if (q == self) continue;
                const double qq = sq_dist<DIM, GENERAL>(a.g, yx, yy, yz, sx[q], sy[q],
                                                        (DIM == 3) ? sz[q] : 0.0);
                double sig2;
                if (POLY) {
                    const double sig = Ri + a.s * srho[q];
                    sig2 = sig * sig;
                } else {
                    sig2 = a.sig2_mono;
                }
                if (qq <= sig2) return true;
            }
        }
    }
    return false;
}

// Phase A, one stencil row of the particle in LDS slot p (own cell [ob, oe)):
// append to nl every candidate of slots [lo, hi) outside the own cell within
// R_i + R_j + 2 c_m of p; *count counts all of them (beyond kNear the list is
// incomplete and phase B scans the whole stencil instead).
template <int DIM, bool POLY, bool GENERAL>
__device__ __forceinline__ void near_row(const PassArgs &a, const double *sx, const double *sy,
                                         const double *sz, const double *srho, int32_t lo,
                                         int32_t hi, int32_t ob, int32_t oe, int32_t p,
                                         uint16_t *nl, int32_t *count)
{
    using C = QuadCfg<DIM, POLY>;
    const double px = sx[p], py = sy[p], pz = (DIM == 3) ? sz[p] : 0.0;
    const double Ri = POLY ? a.s * srho[p] : a.s;
    const double margin = 2.0 * a.c_m;
    for (int32_t c = lo; c < hi; ++c) {
        if (c >= ob && c < oe) continue;
        const double qq = sq_dist<DIM, GENERAL>(a.g, px, py, pz, sx[c], sy[c],
                                                (DIM == 3) ? sz[c] : 0.0);
        const double reach = (POLY ? Ri + a.s * srho[c] : Ri + Ri) + margin;
        if (qq <= reach * reach) {
            const int32_t slot = atomicAdd(count, 1);
            if (slot < C::kNear) nl[slot] = (uint16_t)c;
        }
    }
}

// Phase B test of one trial position y of the particle in LDS slot p.
template <int DIM, bool POLY, bool GENERAL>
__device__ __forceinline__ bool trial_hits(const PassArgs &a, const double *sx, const double *sy,
                                           const double *sz, const double *srho,
                                           const uint16_t *lst, const uint16_t *nl, int32_t nn,
                                           int32_t rx, int32_t ry, int32_t rz, int32_t ob,
                                           int32_t oe, int32_t p, double yx, double yy,
                                           double yz, double Ri)
{
    if (nn == 255)
        return lds_hits<DIM, POLY, GENERAL>(a, sx, sy, sz, srho, lst, rx, ry, rz, p, yx, yy, yz,
                                            Ri);
    for (int32_t e = 0; e < nn; ++e) {
        const int32_t c = nl[e];
        const double qq = sq_dist<DIM, GENERAL>(a.g, yx, yy, yz, sx[c], sy[c],
                                                (DIM == 3) ? sz[c] : 0.0);
        double sig2;
        if (POLY) {
            const double sig = Ri + a.s * srho[c];
            sig2 = sig * sig;
        } else {
            sig2 = a.sig2_mono;
        }
        if (qq <= sig2) return true;
    }
    for (int32_t c = ob; c < oe; ++c) {
        if (c == p) continue;
        const double qq = sq_dist<DIM, GENERAL>(a.g, yx, yy, yz, sx[c], sy[c],
                                                (DIM == 3) ? sz[c] : 0.0);
        double sig2;
        if (POLY) {
            const double sig = Ri + a.s * srho[c];
            sig2 = sig * sig;
        } else {
            sig2 = a.sig2_mono;
        }
        if (qq <= sig2) return true;
    }
    return false;
}

// Does trial position y meet a candidate of the near list (other cells only)?
template <int DIM, bool POLY, bool GENERAL>
__device__ __forceinline__ bool near_hits(const PassArgs &a, const double *sx, const double *sy,
                                          const double *sz, const double *srho,
                                          const uint16_t *nl, int32_t nn, double yx, double yy,
                                          double yz, double Ri)
{
    for (int32_t e = 0; e < nn; ++e) {
        const int32_t c = nl[e];
        const double qq = sq_dist<DIM, GENERAL>(a.g, yx, yy, yz, sx[c], sy[c],
                                                (DIM == 3) ? sz[c] : 0.0);
        double sig2;
        if (POLY) {
            const double sig = Ri + a.s * srho[c];
            sig2 = sig * sig;
        } else {
            sig2 = a.sig2_mono;
        }
        if (qq <= sig2) return true;
    }
    return false;
}

// Does trial position y meet the particle in LDS slot c?
template <int DIM, bool POLY, bool GENERAL>
__device__ __forceinline__ bool slot_hit(const PassArgs &a, const double *sx, const double *sy,
                                         const double *sz, const double *srho, int32_t c,
                                         double yx, double yy, double yz, double Ri)
{
    const double qq = sq_dist<DIM, GENERAL>(a.g, yx, yy, yz, sx[c], sy[c],
                                            (DIM == 3) ? sz[c] : 0.0);
    double sig2;
    if (POLY) {
        const double sig = Ri + a.s * srho[c];
        sig2 = sig * sig;
    } else {
        sig2 = a.sig2_mono;
    }
    return qq <= sig2;
}

template <int DIM, bool POLY, class C>
__device__ __forceinline__ void tile_pass(const PassArgs &a, const TileLattice &L)
{
    __shared__ double sx[C::kCap];
    __shared__ double sy[C::kCap];
    __shared__ double sz[DIM == 3 ? C::kCap : 1];
    __shared__ double srho[POLY ? C::kCap : 1];
    __shared__ uint16_t lst[C::kCells + 1];
    __shared__ uint16_t obase[65];
    __shared__ uint16_t nearl[C::kOwn][C::kNear];
    __shared__ int32_t ncnt[C::kOwn];  // near-list lengths (may exceed kNear: overflow)
    __shared__ uint8_t own_k[C::kOwn];  // own particle -> its own-cell slot (phase A)
    __shared__ int32_t wtot[4];

    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // run of tiles so neighbouring tiles share its L2.
    const int32_t b = blockIdx.x;
    const int32_t tile = (b & 7) * L.per_xcd + (b >> 3);
    if (tile >= L.tiles) return;
    int32_t tx, ty, tz;
    tile_coords<DIM>(L, tile, tx, ty, tz);
    const int tid = threadIdx.x;
    const int32_t na0 = a.g.na[0], na1 = a.g.na[1], na2 = a.g.na[2];
    // global cell of region cell (0, 0, 0): one cell below the tile's first
    const int32_t ox = 2 * C::T * tx + L.off[0] - 1;
    const int32_t oy = 2 * C::T * ty + L.off[1] - 1;
    const int32_t oz = (DIM == 3) ? 2 * C::T * tz + L.off[2] - 1 : 0;

    // 1. particle counts of the region cells (thread owns cells r = kPer*tid + j)
    int32_t gs[C::kPer], cn[C::kPer];
    int32_t mine = 0;
#pragma unroll
    for (int j = 0; j < C::kPer; ++j) {
        const int32_t r = C::kPer * tid + j;
        gs[j] = 0;
        cn[j] = 0;
        if (r < C::kCells) {
            const int32_t rx = r % C::R, ry = (r / C::R) % C::R;
            const int32_t rz = (DIM == 3) ? r / (C::R * C::R) : 0;
            const int32_t gx = wrap_index(ox + rx, na0), gy = wrap_index(oy + ry, na1);
            const int32_t gz = (DIM == 3) ? wrap_index(oz + rz, na2) : 0;
            const int32_t gc = gx + na0 * (gy + na1 * gz);
            gs[j] = a.start[gc];
            cn[j] = a.start[gc + 1] - gs[j];
            mine += cn[j];
        }
    }
    // 2. block exclusive scan -> local CSR starts
    const int32_t inc = wave_inclusive_scan(mine);
    if ((tid & 63) == 63) wtot[tid >> 6] = inc;
    __syncthreads();
    int32_t off = inc - mine, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int32_t t_ = wtot[w];
        if (w < (tid >> 6)) off += t_;
        total += t_;
    }
    if (total > C::kCap) {
        // over capacity: the global-memory kernel takes this tile
        if (tid == 0) {
            const int32_t slot = atomicAdd(&L.ovf[L.colour], 1);
            L.ovf[8 + L.colour * L.max_tiles + slot] = tile;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < C::kPer; ++j) {
        const int32_t r = C::kPer * tid + j;
        if (r < C::kCells) lst[r] = (uint16_t)off;
        off += cn[j];
    }
    if (tid == 0) lst[C::kCells] = (uint16_t)total;

    // 3. stage positions: the first three particles of each of the thread's
    // cells are loaded together (one memory round trip), the rest after
    {
        double vx[C::kPer][3], vy[C::kPer][3], vz[C::kPer][3], vr[C::kPer][3];
#pragma unroll
        for (int j = 0; j < C::kPer; ++j) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (k < cn[j]) {
                    vx[j][k] = a.buf.x[0][gs[j] + k];
                    vy[j][k] = a.buf.x[1][gs[j] + k];
                    if (DIM == 3) vz[j][k] = a.buf.x[2][gs[j] + k];
                    if (POLY) vr[j][k] = a.buf.rho[gs[j] + k];
                }
            }
        }
        int32_t d = off;
#pragma unroll
        for (int j = C::kPer - 1; j >= 0; --j) d -= cn[j];
#pragma unroll
        for (int j = 0; j < C::kPer; ++j) {
            const int32_t d0 = d, g0 = gs[j];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (k < cn[j]) {
                    sx[d0 + k] = vx[j][k];
                    sy[d0 + k] = vy[j][k];
                    if (DIM == 3) sz[d0 + k] = vz[j][k];
                    if (POLY) srho[d0 + k] = vr[j][k];
                }
            }
            for (int32_t k = 3; k < cn[j]; ++k) {
                sx[d0 + k] = a.buf.x[0][g0 + k];
                sy[d0 + k] = a.buf.x[1][g0 + k];
                if (DIM == 3) sz[d0 + k] = a.buf.x[2][g0 + k];
                if (POLY) srho[d0 + k] = a.buf.rho[g0 + k];
            }
            d += cn[j];
        }
    }
    __syncthreads();

    // 4. own cells: slot k of the tile -> particles obase[k] .. obase[k+1]
    const int q = tid >> 2, sub = tid & 3;
    auto own_cell = [&](int k, int32_t &lx_, int32_t &ly_, int32_t &lz_, bool &act_) {
        lx_ = k % C::T;
        ly_ = (k / C::T) % C::T;
        lz_ = (DIM == 3) ? k / (C::T * C::T) : 0;
        act_ = C::T * tx + lx_ < L.h[0] && C::T * ty + ly_ < L.h[1] &&
               (DIM == 2 || C::T * tz + lz_ < L.h[2]);
    };
    auto region_index = [&](int32_t lx_, int32_t ly_, int32_t lz_) {
        return (2 * lx_ + 1) + C::R * ((2 * ly_ + 1) + C::R * ((DIM == 3) ? 2 * lz_ + 1 : 0));
    };
    if (tid < 64) {
        int32_t lx_, ly_, lz_;
        bool act_;
        own_cell(tid, lx_, ly_, lz_, act_);
        const int32_t ro_ = region_index(lx_, ly_, lz_);
        const int32_t m_ = act_ ? (int32_t)lst[ro_ + 1] - (int32_t)lst[ro_] : 0;
        const int32_t incl = wave_inclusive_scan(m_);
        obase[tid] = (uint16_t)(incl - m_);
        if (tid == 63) obase[64] = (uint16_t)(incl > 65535 ? 65535 : incl);
        if (incl <= C::kOwn)
            for (int32_t j = incl - m_; j < incl; ++j) own_k[j] = (uint8_t)tid;
    }
    for (int32_t o = tid; o < C::kOwn; o += 256) ncnt[o] = 0;
    __syncthreads();
    const int32_t nown = obase[64];
    const bool use_near = nown <= C::kOwn;

    // 5. phase A: near lists for every own particle.  One lane per (own
    // particle, stencil row): the row's candidates outside the particle's
    // cell within R_i + R_j + 2 c_m of its old position are appended
    // (LDS atomics; the order of a list does not matter).
    if (use_near) {
        constexpr int kRowsA = Rows<DIM>::kRows;
        for (int32_t w = tid; w < nown * kRowsA; w += 256) {
            const int32_t o = w / kRowsA, row = w - o * kRowsA;
            const int32_t klo = own_k[o];
            int32_t lx_, ly_, lz_;
            bool act_;
            own_cell(klo, lx_, ly_, lz_, act_);
            const int32_t ro_ = region_index(lx_, ly_, lz_);
            const int32_t ob = lst[ro_], oe = lst[ro_ + 1];
            const int32_t p = ob + (o - obase[klo]);
            const int32_t cx_ = 2 * (C::T * tx + lx_) + L.off[0];
            const int32_t cy_ = 2 * (C::T * ty + ly_) + L.off[1];
            const int32_t cz_ = (DIM == 3) ? 2 * (C::T * tz + lz_) + L.off[2] : 0;
            const int32_t rx_ = 2 * lx_ + 1, ry_ = 2 * ly_ + 1, rz_ = (DIM == 3) ? 2 * lz_ + 1 : 0;
            const int32_t iy = row % 3, iz = row / 3;
            const int32_t r0 = (ry_ + iy - 1) * C::R + ((DIM == 3) ? (rz_ + iz - 1) * C::R * C::R : 0);
            const int32_t lo = lst[r0 + rx_ - 1], hi = lst[r0 + rx_ + 2];
            if (is_interior<DIM>(a.g, cx_, cy_, cz_))
                near_row<DIM, POLY, false>(a, sx, sy, sz, srho, lo, hi, ob, oe, p, nearl[o],
                                           &ncnt[o]);
            else
                near_row<DIM, POLY, true>(a, sx, sy, sz, srho, lo, hi, ob, oe, p, nearl[o],
                                          &ncnt[o]);
        }
    }
    __syncthreads();

    // 6. phase B: quad q runs its cell's particles in ascending id order
    int32_t lx, ly, lz;
    bool active;
    own_cell(q, lx, ly, lz, active);
    if (!active) return;
    const int32_t rx = 2 * lx + 1, ry = 2 * ly + 1, rz = (DIM == 3) ? 2 * lz + 1 : 0;
    const int32_t ro = region_index(lx, ly, lz);
    const int32_t ob = lst[ro], oe = lst[ro + 1];
    if (ob == oe) return;
    const int32_t cx = 2 * (C::T * tx + lx) + L.off[0];
    const int32_t cy = 2 * (C::T * ty + ly) + L.off[1];
    const int32_t cz = (DIM == 3) ? 2 * (C::T * tz + lz) + L.off[2] : 0;
    const int32_t gb = a.start[cx + na0 * (cy + na1 * cz)];
    const bool general = !is_interior<DIM>(a.g, cx, cy, cz);
    const int32_t o0 = obase[q];

    // Groups of up to four particles of the cell.  The near list holds only
    // other cells' particles, which no lane moves during this colour phase,
    // so each particle's first trial that meets no near-list candidate can be
    // found before any cell mate settles (trials before it are rejected
    // whatever the cell mates do): lane `sub` draws trial 1 of particle
    // g0 + sub, and for each particle whose trial 1 meets the list the quad
    // draws its later trials four at a time, so no lane waits on another
    // lane's long run of trials.  Then the group is settled in id order: that trial
    // is accepted if it also misses the cell mates at their current
    // positions; otherwise (or without a near list) the quad tests the
    // remaining trials four at a time against the whole neighbourhood.
    // Either way each particle takes its first free trial, in id order.
    for (int32_t g0 = ob; g0 < oe; g0 += 4) {
        const int32_t ps = g0 + sub;
        bool spec = false, pend = false;
        int32_t l1 = 0;  // first near-free trial of particle ps (0: none)
        double sx1 = 0.0, sy1 = 0.0, sz1 = 0.0;
        if (ps < oe) {
            const int32_t o = o0 + (ps - ob);
            spec = use_near && ncnt[o] <= C::kNear;
            if (spec && a.n_l >= 1) {
                const double px = sx[ps], py = sy[ps], pz = (DIM == 3) ? sz[ps] : 0.0;
                const double Ri = POLY ? a.s * srho[ps] : a.s;
                const uint32_t id = (uint32_t)a.buf.id[gb + (ps - ob)];
                Draw d = a.draw;
                double v[3];
                d.word = a.draw.word | (1u << 8);
                unit_vector<DIM>(d, id, 0, a.c_m, v);
                const double yx = wrap_coord(px + v[0], a.g.box[0]);
                const double yy = wrap_coord(py + v[1], a.g.box[1]);
                const double yz = (DIM == 3) ? wrap_coord(pz + v[2], a.g.box[2]) : 0.0;
                const bool hit =
                    general ? near_hits<DIM, POLY, true>(a, sx, sy, sz, srho, nearl[o], ncnt[o],
                                                         yx, yy, yz, Ri)
                            : near_hits<DIM, POLY, false>(a, sx, sy, sz, srho, nearl[o], ncnt[o],
                                                          yx, yy, yz, Ri);
                if (!hit) {
                    l1 = 1;
                    sx1 = yx;
                    sy1 = yy;
                    sz1 = yz;
                } else {
                    pend = a.n_l > 1;
                }
            }
        }
        // Particles whose first trial meets the near list: the quad tests
        // their later trials four at a time, one particle after another.
        for (uint32_t pm = quad_bits(__ballot(pend)); pm != 0; pm &= pm - 1) {
            const int32_t j = __ffs(pm) - 1;
            const int32_t pj = g0 + j;
            const int32_t oj = o0 + (pj - ob);
            const double px = sx[pj], py = sy[pj], pz = (DIM == 3) ? sz[pj] : 0.0;
            const double Rj = POLY ? a.s * srho[pj] : a.s;
            const uint32_t idj = (uint32_t)a.buf.id[gb + (pj - ob)];
            const int32_t nnj = ncnt[oj];
            int32_t found = 0;
            double fx = 0.0, fy = 0.0, fz = 0.0;
            Draw d = a.draw;
            for (int32_t base = 2; base <= a.n_l; base += 4) {
                const int32_t l = base + sub;
                bool free_ = false;
                double yx = 0.0, yy = 0.0, yz = 0.0;
                if (l <= a.n_l) {
                    double v[3];
                    d.word = a.draw.word | ((uint32_t)l << 8);
                    unit_vector<DIM>(d, idj, 0, a.c_m, v);
                    yx = wrap_coord(px + v[0], a.g.box[0]);
                    yy = wrap_coord(py + v[1], a.g.box[1]);
                    yz = (DIM == 3) ? wrap_coord(pz + v[2], a.g.box[2]) : 0.0;
                    free_ = !(general ? near_hits<DIM, POLY, true>(a, sx, sy, sz, srho, nearl[oj],
                                                                   nnj, yx, yy, yz, Rj)
                                      : near_hits<DIM, POLY, false>(a, sx, sy, sz, srho,
                                                                    nearl[oj], nnj, yx, yy, yz,
                                                                    Rj));
                }
                const uint32_t fb = quad_bits(__ballot(free_));
                if (fb) {
                    const int win = __ffs(fb) - 1;
                    const int32_t src = (tid & 63 & ~3) | win;
                    found = base + win;
                    fx = __shfl(yx, src, 64);
                    fy = __shfl(yy, src, 64);
                    fz = __shfl(yz, src, 64);
                    break;
                }
            }
            if (sub == j) {
                l1 = found;
                sx1 = fx;
                sy1 = fy;
                sz1 = fz;
            }
        }
        const int32_t gend = (oe - g0 < 4) ? oe : g0 + 4;
        for (int32_t p = g0; p < gend; ++p) {
            const int32_t src = (tid & 63 & ~3) | (p - g0);
            const bool sp = __shfl((int)spec, src, 64) != 0;
            const int32_t lp = __shfl(l1, src, 64);
            const double qx = __shfl(sx1, src, 64);
            const double qy = __shfl(sy1, src, 64);
            const double qz = __shfl(sz1, src, 64);
            const int32_t gp = gb + (p - ob);
            const double Ri = POLY ? a.s * srho[p] : a.s;
            uint8_t code = 0;
            int32_t first = 1;
            bool done = false;
            if (sp) {
                if (lp == 0) {
                    done = true;  // every trial meets the near list
                } else {
                    bool hit = false;
                    for (int32_t c = ob + sub; c < oe; c += 4) {
                        if (c == p) continue;
                        hit = hit || (general ? slot_hit<DIM, POLY, true>(a, sx, sy, sz, srho, c,
                                                                          qx, qy, qz, Ri)
                                              : slot_hit<DIM, POLY, false>(a, sx, sy, sz, srho, c,
                                                                           qx, qy, qz, Ri));
                    }
                    if (quad_bits(__ballot(hit)) == 0) {
                        done = true;
                        code = (uint8_t)lp;
                        if (sub == 0) {
                            sx[p] = qx;
                            sy[p] = qy;
                            if (DIM == 3) sz[p] = qz;
                            a.buf.x[0][gp] = qx;
                            a.buf.x[1][gp] = qy;
                            if (DIM == 3) a.buf.x[2][gp] = qz;
                        }
                    } else {
                        first = lp + 1;
                    }
                }
            }
            if (!done) {
                const int32_t o = o0 + (p - ob);
                const double px = sx[p], py = sy[p], pz = (DIM == 3) ? sz[p] : 0.0;
                const int32_t nn = use_near ? (ncnt[o] > C::kNear ? 255 : ncnt[o]) : 255;
                const uint16_t *nl = use_near ? nearl[o] : nullptr;
                const uint32_t id = (uint32_t)a.buf.id[gp];
                Draw d = a.draw;
                for (int32_t base = first; base <= a.n_l; base += 4) {
                    const int32_t l = base + sub;
                    bool free_ = false;
                    double yx = 0.0, yy = 0.0, yz = 0.0;
                    if (l <= a.n_l) {
                        double v[3];
                        d.word = a.draw.word | ((uint32_t)l << 8);
                        unit_vector<DIM>(d, id, 0, a.c_m, v);
                        yx = wrap_coord(px + v[0], a.g.box[0]);
                        yy = wrap_coord(py + v[1], a.g.box[1]);
                        yz = (DIM == 3) ? wrap_coord(pz + v[2], a.g.box[2]) : 0.0;
                        const bool hit =
                            general ? trial_hits<DIM, POLY, true>(a, sx, sy, sz, srho, lst, nl, nn,
                                                                  rx, ry, rz, ob, oe, p, yx, yy,
                                                                  yz, Ri)
                                    : trial_hits<DIM, POLY, false>(a, sx, sy, sz, srho, lst, nl,
                                                                   nn, rx, ry, rz, ob, oe, p, yx,
                                                                   yy, yz, Ri);
                        free_ = !hit;
                    }
                    const uint32_t fb = quad_bits(__ballot(free_));
                    if (fb) {
                        const int win = __ffs(fb) - 1;
                        if (sub == win) {
                            sx[p] = yx;
                            sy[p] = yy;
                            if (DIM == 3) sz[p] = yz;
                            a.buf.x[0][gp] = yx;
                            a.buf.x[1][gp] = yy;
                            if (DIM == 3) a.buf.x[2][gp] = yz;
                        }
                        code = (uint8_t)(base + win);
                        break;
                    }
                }
            }
            if (sub == 0) {
                a.acc[gp] = code;
                if (code == 0) a.failed[1 + atomicAdd(&a.failed[0], 1)] = gp;
            }
            // the accepted position in LDS must be seen by the next particle
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

template <int DIM, bool POLY>
__global__ void __launch_bounds__(256) k_migrate_tile(PassArgs a, TileLattice L)
{
    tile_pass<DIM, POLY, QuadCfg<DIM, POLY>>(a, L);
}

// The same pass with a larger LDS region (denser grids, 3D).
template <int DIM, bool POLY>
__global__ void __launch_bounds__(256) k_migrate_tile_wide(PassArgs a, TileLattice L)
{
    tile_pass<DIM, POLY, QuadCfg<DIM, POLY, 2>>(a, L);
}

// A middle region (3D, three workgroups a CU).
template <int DIM, bool POLY>
__global__ void __launch_bounds__(256) k_migrate_tile_mid(PassArgs a, TileLattice L)
{
    tile_pass<DIM, POLY, QuadCfg<DIM, POLY, 1>>(a, L);
}

// Tiles queued by k_migrate_tile because their neighbourhood exceeds LDS:
// one thread per colour cell, candidates read from global memory.
template <int DIM, bool POLY>
__global__ void __launch_bounds__(64) k_migrate_overflow(PassArgs a, TileLattice L)
{
    using C = QuadCfg<DIM, POLY>;
    const int32_t count = L.ovf[L.colour];
    const int32_t *list = L.ovf + 8 + L.colour * L.max_tiles;
    for (int32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int32_t tile = list[i];
        int32_t tx, ty, tz;
        tile_coords<DIM>(L, tile, tx, ty, tz);
        const int q = threadIdx.x;
        const int32_t lx = q % C::T, ly = (q / C::T) % C::T;
        const int32_t lz = (DIM == 3) ? q / (C::T * C::T) : 0;
        const int32_t jx = C::T * tx + lx, jy = C::T * ty + ly;
        const int32_t jz = (DIM == 3) ? C::T * tz + lz : 0;
        if (jx < L.h[0] && jy < L.h[1] && (DIM == 2 || jz < L.h[2]))
            migrate_cell_global<DIM, POLY>(a, 2 * jx + L.off[0], 2 * jy + L.off[1],
                                           (DIM == 3) ? 2 * jz + L.off[2] : 0);
    }
}

// Algorithm 6 after a pass: some pair overlaps iff some particle that
// rejected all of its trials overlaps another one (a particle that accepted
// a trial was tested against every particle processed before it at its final
// position and every later one at a position it kept if it was rejected).
// So only particles with accept code 0 are tested; check_all tests every
// particle (initial-state validation).
// The same check with one wavefront per failed particle (crowded cells).
template <int DIM, bool POLY>
__global__ void __launch_bounds__(kBlock) k_check_ball_wave(PassArgs a, Counters *cnt)
{
    const int32_t count = a.failed[0];
    const int lane = threadIdx.x & 63;
    const int32_t waves = gridDim.x * (kBlock / 64);
    for (int32_t i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); i < count; i += waves) {
        if (__atomic_load_n(&cnt->overlap, __ATOMIC_RELAXED)) return;  // already known
        if (check_ball_wave<DIM, POLY>(a, a.failed[1 + i], lane) && lane == 0)
            atomicOr(&cnt->overlap, 1);
    }
}

template <int DIM, bool POLY>
__global__ void __launch_bounds__(kBlock) k_check_ball(PassArgs a, int32_t check_all, Counters *cnt)
{
    const int32_t count = check_all ? a.n : a.failed[0];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += gridDim.x * blockDim.x) {
        const int32_t p = check_all ? i : a.failed[1 + i];
        if (check_ball_one<DIM, POLY>(a, p)) atomicOr(&cnt->overlap, 1);
    }
}

// The same check on the failed list with kCheckGroup lanes per particle:
// one lane's scan of the stencil is a chain of some fifty dependent global
// loads, so the lanes of a group split the candidates (the same exact test
// as check_ball_one; any lane's hit sets the flag).
constexpr int kCheckGroup = 8;

template <int DIM, bool POLY>
__global__ void __launch_bounds__(kBlock) k_check_ball_group(PassArgs a, Counters *cnt)
{
    const int32_t count = a.failed[0];
    const int sub = threadIdx.x & (kCheckGroup - 1);
    const int32_t groups = (int32_t)(gridDim.x * blockDim.x / kCheckGroup);
    const double *__restrict__ X = a.buf.x[0];
    const double *__restrict__ Y = a.buf.x[1];
    const double *__restrict__ Z = a.buf.x[2];
    for (int32_t i = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / kCheckGroup); i < count;
         i += groups) {
        const int32_t p = a.failed[1 + i];
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
            for (int32_t q = lo[r] + sub; q < hi[r] && !hit; q += kCheckGroup) {
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
        if (hit) atomicOr(&cnt->overlap, 1);
    }
}


// ---------------------------------------------------------------- platelets

// Thin platelets (3D): the trial moves the centre by c_m times a random
// unit vector (stream 0) and the normal to (n + c_n w) / |n + c_n w| (w a
// random unit vector, stream 1); both are accepted or rejected together.
// The pair test is the exact disk-disk intersection (zero thickness) or
// the spherodisk test (platelets_touch), with the lower id as disk 1.
template <bool SD>
__device__ __forceinline__ bool platelet_hits(const PassArgs &a, const int32_t *lo,
                                              const int32_t *hi, int32_t self, int32_t self_id,
                                              double yx, double yy, double yz, const double ny[3],
                                              double ai)
{
    const double *__restrict__ X = a.buf.x[0];
    const double *__restrict__ Y = a.buf.x[1];
    const double *__restrict__ Z = a.buf.x[2];
#pragma unroll
    for (int r = 0; r < Rows<3>::kRanges; ++r) {
        for (int32_t q = lo[r]; q < hi[r]; ++q) {
            if (q == self) continue;
            const double aj = a.buf.rho ? a.s * a.buf.rho[q] : a.s;
            const double nq[3] = {a.buf.nrm[0][q], a.buf.nrm[1][q], a.buf.nrm[2][q]};
            const int32_t qid = a.buf.id[q];
            bool hit;
            if (self_id < qid) {
                const double dx = min_image(X[q] - yx, a.g.box[0], a.g.half[0]);
                const double dy = min_image(Y[q] - yy, a.g.box[1], a.g.half[1]);
                const double dz = min_image(Z[q] - yz, a.g.box[2], a.g.half[2]);
                hit = platelets_touch<SD>(dx, dy, dz, ny, ai, nq, aj, a.tau);
            } else {
                const double dx = min_image(yx - X[q], a.g.box[0], a.g.half[0]);
                const double dy = min_image(yy - Y[q], a.g.box[1], a.g.half[1]);
                const double dz = min_image(yz - Z[q], a.g.box[2], a.g.half[2]);
                hit = platelets_touch<SD>(dx, dy, dz, nq, aj, ny, ai, a.tau);
            }
            if (hit) return true;
        }
    }
    return false;
}

template <bool SD>
__device__ void migrate_platelet_cell(const PassArgs &a, int32_t cx, int32_t cy, int32_t cz);

// Platelets on crowded grids: one 64-lane wavefront per colour cell, the
// scheme of migrate_cell_wave.  A disk meets another only if their centres
// are within a_i + a_j, so the near lists are built on centre distance
// (+ 2 c_m for candidates outside the cell, + 3 c_m for cell mates) and the
// lanes split (trial, near entry) pairs, each running the exact disk-disk
// test with the lower id as disk 1.
constexpr int kPlateOwn = 64;
// Near-list capacities: 32 entries, or 96 when large migration steps put
// tens of disks within reach (chosen per pass on the host).
constexpr int kPlateNearShort = 32;
constexpr int kPlateNearLong = 96;

struct PlateOwn {
    double x, y, z, a, n0, n1, n2;
    int32_t id, pad;
};

template <int NEAR>
struct PlateLds {
    PlateOwn own[kPlateOwn];
    float4 own32[kPlateOwn];  // centre and radius rounded to FP32, for the near-list filter
    int32_t nn[kPlateOwn];
    int32_t near[kPlateOwn * NEAR];  // slot q >= 0, or -(k + 1) for own particle k
    int32_t nfail;
    int32_t fail[kPlateOwn];  // own indices that rejected every trial
};

// Trial l of a platelet: centre (stream 0, length c_m, wrapped) and normal
// (stream 1: (n + c_n w) / |n + c_n w|).
__device__ __forceinline__ void plate_trial(const PassArgs &a, const PlateOwn &me, int32_t l,
                                            double y[3], double ny[3])
{
    Draw d = a.draw;
    d.word = a.draw.word | ((uint32_t)l << 8);
    double v[3], w[3];
    unit_vector<3>(d, (uint32_t)me.id, 0, a.c_m, v);
    y[0] = wrap_coord(me.x + v[0], a.g.box[0]);
    y[1] = wrap_coord(me.y + v[1], a.g.box[1]);
    y[2] = wrap_coord(me.z + v[2], a.g.box[2]);
    unit_vector<3>(d, (uint32_t)me.id, 1, a.c_n, w);
    const double m0 = me.n0 + w[0], m1 = me.n1 + w[1], m2 = me.n2 + w[2];
    const double mm = m0 * m0 + m1 * m1 + m2 * m2;
    const double inv = 1.0 / __builtin_sqrt(mm);
    ny[0] = m0 * inv;
    ny[1] = m1 * inv;
    ny[2] = m2 * inv;
}

// The exact pair test of platelet_hits for one candidate.
template <bool SD>
__device__ __forceinline__ bool plate_pair_hit(const PassArgs &a, int32_t self_id, const double y[3],
                                               const double ny[3], double ai, double qx, double qy,
                                               double qz, const double nq[3], double aj,
                                               int32_t qid)
{
    if (self_id < qid) {
        const double dx = min_image(qx - y[0], a.g.box[0], a.g.half[0]);
        const double dy = min_image(qy - y[1], a.g.box[1], a.g.half[1]);
        const double dz = min_image(qz - y[2], a.g.box[2], a.g.half[2]);
        return platelets_touch<SD>(dx, dy, dz, ny, ai, nq, aj, a.tau);
    }
    const double dx = min_image(y[0] - qx, a.g.box[0], a.g.half[0]);
    const double dy = min_image(y[1] - qy, a.g.box[1], a.g.half[1]);
    const double dz = min_image(y[2] - qz, a.g.box[2], a.g.half[2]);
    return platelets_touch<SD>(dx, dy, dz, nq, aj, ny, ai, a.tau);
}

template <bool SD, class LDS>
__device__ __forceinline__ bool plate_ref_hit(const PassArgs &a, const LDS &L, int32_t ref,
                                              int32_t self_id, const double y[3],
                                              const double ny[3], double ai)
{
    if (ref < 0) {
        const PlateOwn o = L.own[-ref - 1];
        const double nq[3] = {o.n0, o.n1, o.n2};
        return plate_pair_hit<SD>(a, self_id, y, ny, ai, o.x, o.y, o.z, nq, o.a, o.id);
    }
    const double nq[3] = {a.buf.nrm[0][ref], a.buf.nrm[1][ref], a.buf.nrm[2][ref]};
    const double aj = a.buf.rho ? a.s * a.buf.rho[ref] : a.s;
    return plate_pair_hit<SD>(a, self_id, y, ny, ai, a.buf.x[0][ref], a.buf.x[1][ref],
                          a.buf.x[2][ref], nq, aj, a.buf.id[ref]);
}

// Algorithm 3 for the platelets of one cell (global-memory path, one thread).
template <bool SD>
__device__ void migrate_platelet_cell(const PassArgs &a, int32_t cx, int32_t cy, int32_t cz)
{
    const int32_t c = cx + a.g.na[0] * (cy + a.g.na[1] * cz);
    const int32_t beg = a.start[c], end = a.start[c + 1];
    if (beg == end) return;
    int32_t lo[Rows<3>::kRanges], hi[Rows<3>::kRanges];
    stencil_slices<3>(a.g, a.start, cx, cy, cz, lo, hi);
    double *__restrict__ X = a.buf.x[0];
    double *__restrict__ Y = a.buf.x[1];
    double *__restrict__ Z = a.buf.x[2];
    for (int32_t p = beg; p < end; ++p) {
        const double ox = X[p], oy = Y[p], oz = Z[p];
        const double n0 = a.buf.nrm[0][p], n1 = a.buf.nrm[1][p], n2 = a.buf.nrm[2][p];
        const int32_t pid = a.buf.id[p];
        const double ai = a.buf.rho ? a.s * a.buf.rho[p] : a.s;
        uint8_t code = 0;
        Draw d = a.draw;
        for (int32_t l = 1; l <= a.n_l; ++l) {
            d.word = a.draw.word | ((uint32_t)l << 8);
            double v[3], w[3];
            unit_vector<3>(d, (uint32_t)pid, 0, a.c_m, v);
            const double yx = wrap_coord(ox + v[0], a.g.box[0]);
            const double yy = wrap_coord(oy + v[1], a.g.box[1]);
            const double yz = wrap_coord(oz + v[2], a.g.box[2]);
            unit_vector<3>(d, (uint32_t)pid, 1, a.c_n, w);
            const double m0 = n0 + w[0], m1 = n1 + w[1], m2 = n2 + w[2];
            const double mm = m0 * m0 + m1 * m1 + m2 * m2;
            const double inv = 1.0 / __builtin_sqrt(mm);
            const double ny[3] = {m0 * inv, m1 * inv, m2 * inv};
            if (!platelet_hits<SD>(a, lo, hi, p, pid, yx, yy, yz, ny, ai)) {
                X[p] = yx;
                Y[p] = yy;
                Z[p] = yz;
                a.buf.nrm[0][p] = ny[0];
                a.buf.nrm[1][p] = ny[1];
                a.buf.nrm[2][p] = ny[2];
                code = (uint8_t)l;
                break;
            }
        }
        a.acc[p] = code;
        if (code == 0) a.failed[1 + atomicAdd(&a.failed[0], 1)] = p;
    }
}

template <int NEAR, bool SD>
__global__ void __launch_bounds__(64) k_migrate_platelet_wave(PassArgs a, ColourLattice L)
{
    __shared__ PlateLds<NEAR> S;
    const int lane = threadIdx.x;
    const int32_t t = blockIdx.x;
    const int32_t jx = t % L.h[0];
    const int32_t r1 = t / L.h[0];
    const int32_t jy = r1 % L.h[1];
    const int32_t jz = r1 / L.h[1];
    const int32_t cx = 2 * jx + L.off[0];
    const int32_t cy = 2 * jy + L.off[1];
    const int32_t cz = 2 * jz + L.off[2];
    const int32_t c = cx + a.g.na[0] * (cy + a.g.na[1] * cz);
    const int32_t beg = a.start[c], end = a.start[c + 1];
    const int32_t cnt = end - beg;
    if (cnt == 0) return;
    if (cnt > kPlateOwn) {
        if (lane == 0) migrate_platelet_cell<SD>(a, cx, cy, cz);
        return;
    }
    int32_t lo[Rows<3>::kRanges], hi[Rows<3>::kRanges];
    stencil_slices<3>(a.g, a.start, cx, cy, cz, lo, hi);
    for (int32_t k = lane; k < cnt; k += 64) {
        const int32_t q = beg + k;
        PlateOwn o;
        o.x = a.buf.x[0][q];
        o.y = a.buf.x[1][q];
        o.z = a.buf.x[2][q];
        o.a = a.buf.rho ? a.s * a.buf.rho[q] : a.s;
        o.n0 = a.buf.nrm[0][q];
        o.n1 = a.buf.nrm[1][q];
        o.n2 = a.buf.nrm[2][q];
        o.id = a.buf.id[q];
        o.pad = 0;
        S.own[k] = o;
        S.own32[k] = make_float4((float)o.x, (float)o.y, (float)o.z, (float)o.a);
        S.nn[k] = 0;
    }
    if (lane == 0) S.nfail = 0;
    __syncthreads();
    // A. near lists on centre distance.  A list only has to contain every
    // disk that can meet a trial (the exact FP64 disk test decides later), so
    // the filter runs in FP32 with a margin covering rounding (positions off
    // by at most L 2^-24 each): 4e-7 Lmax absolute plus 1e-5 relative.
    const float bx32 = (float)a.g.box[0], by32 = (float)a.g.box[1], bz32 = (float)a.g.box[2];
    const float hx32 = 0.5f * bx32, hy32 = 0.5f * by32, hz32 = 0.5f * bz32;
    float lmax32 = bx32 > by32 ? bx32 : by32;
    lmax32 = lmax32 > bz32 ? lmax32 : bz32;
    const float tol32 = 4e-7f * lmax32;
    auto near32 = [&](const float4 &o, float px, float py, float pz, float reach) {
        float dx = o.x - px, dy = o.y - py, dz = o.z - pz;
        if (dx > hx32) dx -= bx32;
        if (dx < -hx32) dx += bx32;
        if (dy > hy32) dy -= by32;
        if (dy < -hy32) dy += by32;
        if (dz > hz32) dz -= bz32;
        if (dz < -hz32) dz += bz32;
        const float rr = reach * 1.00001f + tol32;
        return (dx * dx + dy * dy) + dz * dz <= rr * rr;
    };
    const float cm2 = (float)(2.0 * a.c_m), cm3 = (float)(3.0 * a.c_m);
#pragma unroll
    for (int r = 0; r < Rows<3>::kRanges; ++r) {
        for (int32_t q = lo[r] + lane; q < hi[r]; q += 64) {
            if (q >= beg && q < end) continue;
            const float qx = (float)a.buf.x[0][q], qy = (float)a.buf.x[1][q];
            const float qz = (float)a.buf.x[2][q];
            const float aq = (float)(a.buf.rho ? a.s * a.buf.rho[q] : a.s);
            for (int32_t k = 0; k < cnt; ++k) {
                const float4 o = S.own32[k];
                if (near32(o, qx, qy, qz, (o.w + aq) + cm2)) {
                    const int32_t slot = atomicAdd(&S.nn[k], 1);
                    if (slot < NEAR) S.near[k * NEAR + slot] = q;
                }
            }
        }
    }
    for (int32_t j = lane; j < cnt; j += 64) {
        const float4 b = S.own32[j];
        for (int32_t k = 0; k < cnt; ++k) {
            if (k == j) continue;
            const float4 o = S.own32[k];
            if (near32(o, b.x, b.y, b.z, (o.w + b.w) + cm3)) {
                const int32_t slot = atomicAdd(&S.nn[k], 1);
                if (slot < NEAR) S.near[k * NEAR + slot] = -(j + 1);
            }
        }
    }
    __syncthreads();
    // B. the sequential part
    for (int32_t k = 0; k < cnt; ++k) {
        const int32_t p = beg + k;
        const PlateOwn me = S.own[k];
        const int32_t m = S.nn[k];
        int32_t code = 0;
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0;
        // (trial, entry) groups while the list fits its capacity and the lanes
        if (m <= (NEAR < 64 ? NEAR : 64)) {
            const int32_t mm = m > 0 ? m : 1;
            const int32_t G = 64 / mm;
            const int32_t g = lane / mm, j = lane - g * mm;
            const unsigned long long seg = (mm == 64) ? ~0ull : ((1ull << mm) - 1ull);
            for (int32_t l0 = 1; l0 <= a.n_l && code == 0; l0 += G) {
                const int32_t l = l0 + g;
                const bool active = g < G && l <= a.n_l;
                double y[3], ny[3];
                plate_trial(a, me, active ? l : l0, y, ny);
                const bool hit = active && m > 0 &&
                                 plate_ref_hit<SD>(a, S, S.near[k * NEAR + j], me.id, y, ny, me.a);
                const unsigned long long hits = __ballot(hit);
                int32_t win = -1;
                for (int32_t gg = 0; gg < G && l0 + gg <= a.n_l; ++gg) {
                    if (((hits >> (gg * mm)) & seg) == 0) {
                        win = gg;
                        break;
                    }
                }
                if (win >= 0) {
                    code = l0 + win;
                    w0 = __shfl(y[0], win * mm, 64);
                    w1 = __shfl(y[1], win * mm, 64);
                    w2 = __shfl(y[2], win * mm, 64);
                    v0 = __shfl(ny[0], win * mm, 64);
                    v1 = __shfl(ny[1], win * mm, 64);
                    v2 = __shfl(ny[2], win * mm, 64);
                }
            }
        } else if (m <= NEAR) {
            // a long near list: one trial at a time, the lanes split the list
            for (int32_t l = 1; l <= a.n_l && code == 0; ++l) {
                double y[3], ny[3];
                plate_trial(a, me, l, y, ny);
                bool hit = false;
                for (int32_t e = lane; e < m; e += 64)
                    hit = hit || plate_ref_hit<SD>(a, S, S.near[k * NEAR + e], me.id, y, ny, me.a);
                if (__ballot(hit) == 0) {
                    code = l;
                    w0 = y[0];
                    w1 = y[1];
                    w2 = y[2];
                    v0 = ny[0];
                    v1 = ny[1];
                    v2 = ny[2];
                }
            }
        } else {
            // near list overflowed: the whole stencil, one trial at a time
            for (int32_t l = 1; l <= a.n_l && code == 0; ++l) {
                double y[3], ny[3];
                plate_trial(a, me, l, y, ny);
                bool hit = false;
#pragma unroll
                for (int r = 0; r < Rows<3>::kRanges; ++r) {
                    for (int32_t q = lo[r] + lane; q < hi[r]; q += 64) {
                        if (q >= beg && q < end) continue;
                        hit = hit || plate_ref_hit<SD>(a, S, q, me.id, y, ny, me.a);
                    }
                }
                for (int32_t j = lane; j < cnt; j += 64)
                    if (j != k) hit = hit || plate_ref_hit<SD>(a, S, -(j + 1), me.id, y, ny, me.a);
                if (__ballot(hit) == 0) {
                    code = l;
                    w0 = y[0];
                    w1 = y[1];
                    w2 = y[2];
                    v0 = ny[0];
                    v1 = ny[1];
                    v2 = ny[2];
                }
            }
        }
        if (lane == 0) {
            if (code) {
                S.own[k].x = w0;
                S.own[k].y = w1;
                S.own[k].z = w2;
                S.own[k].n0 = v0;
                S.own[k].n1 = v1;
                S.own[k].n2 = v2;
                a.buf.x[0][p] = w0;
                a.buf.x[1][p] = w1;
                a.buf.x[2][p] = w2;
                a.buf.nrm[0][p] = v0;
                a.buf.nrm[1][p] = v1;
                a.buf.nrm[2][p] = v2;
            }
            a.acc[p] = (uint8_t)code;
            if (code == 0) S.fail[S.nfail++] = k;
        }
        // The workgroup is this one wavefront, whose LDS operations complete
        // in order: lane 0's stores only need to be ordered before the next
        // particle's loads (a workgroup barrier would also wait for its
        // global stores on every particle).
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the cell's failures go to the global list once, off the chain
    const int32_t nf = S.nfail;
    if (nf > 0) {
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&a.failed[0], nf);
        base = __shfl(base, 0, 64);
        for (int32_t i = lane; i < nf; i += 64) a.failed[1 + base + i] = beg + S.fail[i];
    }
}

template <bool SD>
__device__ __forceinline__ bool check_platelet_one(const PassArgs &a, int32_t p)
{
    const double x = a.buf.x[0][p], y = a.buf.x[1][p], z = a.buf.x[2][p];
    const double np_[3] = {a.buf.nrm[0][p], a.buf.nrm[1][p], a.buf.nrm[2][p]};
    const int32_t cx = cell_coord(x, a.g.inv_w[0], a.g.na[0]);
    const int32_t cy = cell_coord(y, a.g.inv_w[1], a.g.na[1]);
    const int32_t cz = cell_coord(z, a.g.inv_w[2], a.g.na[2]);
    int32_t lo[Rows<3>::kRanges], hi[Rows<3>::kRanges];
    stencil_slices<3>(a.g, a.start, cx, cy, cz, lo, hi);
    const double ai = a.buf.rho ? a.s * a.buf.rho[p] : a.s;
    return platelet_hits<SD>(a, lo, hi, p, a.buf.id[p], x, y, z, np_, ai);
}

template <bool SD>
__global__ void __launch_bounds__(kBlock) k_check_platelet(PassArgs a, int32_t check_all,
                                                           Counters *cnt)
{
    const int32_t count = check_all ? a.n : a.failed[0];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += gridDim.x * blockDim.x) {
        const int32_t p = check_all ? i : a.failed[1 + i];
        if (check_platelet_one<SD>(a, p)) atomicOr(&cnt->overlap, 1);
    }
}

inline unsigned blocks_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b > 0 ? b : 1);
}

bool colour_lattice(int dim, const Grid &g, int colour, ColourLattice &L)
{
    L.count = 1;
    for (int ax = 0; ax < 3; ++ax) {
        const int bit = (colour >> ax) & 1;
        if (ax < dim && g.na[ax] >= 4) {
            L.h[ax] = g.na[ax] / 2;
            L.off[ax] = bit;
        } else {
            if (bit) return false;
            L.h[ax] = 1;
            L.off[ax] = 0;
        }
        L.count *= L.h[ax];
    }
    return L.count > 0;
}

// The tiled kernel needs at least 2T+1 distinct cells on every axis so that
// a region never holds a cell twice.
bool tile_ok(int dim, const Grid &g)
{
    const int need = (dim == 3) ? 9 : 17;
    for (int ax = 0; ax < dim; ++ax)
        if (g.na[ax] < need) return false;
    return true;
}

}  // namespace

// Crowded grids (mean occupancy of at least kWaveOccupancy particles per
// cell) migrate with one wavefront per cell.
bool wave_cells(int dim, const Grid &g, int32_t n)
{
    int64_t ncell = 1;
    for (int ax = 0; ax < dim; ++ax) ncell *= g.na[ax];
    return (int64_t)n >= (int64_t)kWaveOccupancy * ncell;
}

namespace {

// The tiled kernels stage a tile's (2T+1)^d region in LDS.  A grid takes
// the standard kernel (0) while its mean region load stays below the LDS
// capacity less three Poisson deviations (the counts of a dense hard-sphere
// configuration fluctuate far less than Poisson's), else the middle (1)
// or the wide (2) region (3D) under the same rule, else (3) one wavefront
// per cell: above that load many tiles would fall back to the
// one-thread-per-cell global kernel.
int tile_class(int dim, bool poly, const Grid &g, int32_t n)
{
    double cells = 1.0;
    for (int ax = 0; ax < dim; ++ax) cells *= (double)g.na[ax];
    auto fits = [&](double region, double cap) {
        return (double)n / cells * region <= cap - 3.0 * sqrt(cap);
    };
    if (dim == 3) {
        constexpr double region = QuadCfg<3, false>::kCells;
        if (fits(region, poly ? QuadCfg<3, true>::kCap : QuadCfg<3, false>::kCap)) return 0;
        if (fits(region, poly ? QuadCfg<3, true, 1>::kCap : QuadCfg<3, false, 1>::kCap)) return 1;
        if (fits(region, poly ? QuadCfg<3, true, 2>::kCap : QuadCfg<3, false, 2>::kCap)) return 2;
        return 3;
    }
    constexpr double region = QuadCfg<2, false>::kCells;
    return fits(region, poly ? QuadCfg<2, true>::kCap : QuadCfg<2, false>::kCap) ? 0 : 3;
}

}  // namespace

hipError_t migrate_colour(int dim, int shape, bool poly, const PassArgs &a, int colour,
                          hipStream_t stream, bool *launched, hipEvent_t after_main, int *which)
{
    ColourLattice L;
    *launched = false;
    if (!colour_lattice(dim, a.g, colour, L)) return hipSuccess;
    auto main_done = [&](int kind) {
        if (after_main) (void)hipEventRecord(after_main, stream);
        if (which) *which = kind;
        *launched = true;
    };
    // Sparse ball grids large enough to tile run the LDS-tiled kernels
    // (standard or wide region by the mean load).  Grids too small to tile
    // have few cells per colour phase, where one thread per cell would leave
    // the chip idle behind chains of dependent global loads: they, crowded
    // grids and platelets run one wavefront per cell.
    bool use_tile = shape != SRM_PLATELET && a.ovf && tile_ok(dim, a.g) && !wave_cells(dim, a.g, a.n);
    int tclass = 0;
    TileLattice T{};
    if (use_tile) {
        tclass = tile_class(dim, poly, a.g, a.n);
        const int tsz = (dim == 3) ? 4 : 8;
        T.tiles = 1;
        for (int ax = 0; ax < 3; ++ax) {
            T.h[ax] = L.h[ax];
            T.off[ax] = L.off[ax];
            T.nt[ax] = (ax < dim) ? (L.h[ax] + tsz - 1) / tsz : 1;
            T.tiles *= T.nt[ax];
        }
        use_tile = tclass < 3 && T.tiles <= a.ovf_max_tiles;
    }
    if (use_tile) {
        T.per_xcd = (T.tiles + 7) / 8;
        T.colour = colour;
        T.ovf = a.ovf;
        T.max_tiles = a.ovf_max_tiles;
        const dim3 grid(8 * T.per_xcd), block(256);
        const dim3 ogrid(T.tiles < 512 ? T.tiles : 512), oblock(64);
        if (dim == 3 && tclass == 2) {
            if (poly) hipLaunchKernelGGL((k_migrate_tile_wide<3, true>), grid, block, 0, stream, a, T);
            else hipLaunchKernelGGL((k_migrate_tile_wide<3, false>), grid, block, 0, stream, a, T);
        } else if (dim == 3 && tclass == 1) {
            if (poly) hipLaunchKernelGGL((k_migrate_tile_mid<3, true>), grid, block, 0, stream, a, T);
            else hipLaunchKernelGGL((k_migrate_tile_mid<3, false>), grid, block, 0, stream, a, T);
        } else if (dim == 3) {
            if (poly) hipLaunchKernelGGL((k_migrate_tile<3, true>), grid, block, 0, stream, a, T);
            else hipLaunchKernelGGL((k_migrate_tile<3, false>), grid, block, 0, stream, a, T);
        } else {
            if (poly) hipLaunchKernelGGL((k_migrate_tile<2, true>), grid, block, 0, stream, a, T);
            else hipLaunchKernelGGL((k_migrate_tile<2, false>), grid, block, 0, stream, a, T);
        }
        main_done(tclass == 2 ? SRM_KERNEL_TILE_WIDE : tclass == 1 ? SRM_KERNEL_TILE_MID : SRM_KERNEL_TILE);
        // tiles whose neighbourhood did not fit LDS
        if (dim == 3) {
            if (poly) hipLaunchKernelGGL((k_migrate_overflow<3, true>), ogrid, oblock, 0, stream, a, T);
            else hipLaunchKernelGGL((k_migrate_overflow<3, false>), ogrid, oblock, 0, stream, a, T);
        } else {
            if (poly) hipLaunchKernelGGL((k_migrate_overflow<2, true>), ogrid, oblock, 0, stream, a, T);
            else hipLaunchKernelGGL((k_migrate_overflow<2, false>), ogrid, oblock, 0, stream, a, T);
        }
        return hipGetLastError();
    }
    const dim3 grid(L.count), block(64);
    if (shape == SRM_PLATELET) {
        // expected near-list length: centres within 2 s + 2 c_m at the mean
        // density (s the radius scale; unequal platelets may overflow the
        // short list, which only costs time)
        const double reach = 2.0 * a.s + 2.0 * a.c_m;
        const double vol = a.g.box[0] * a.g.box[1] * a.g.box[2];
        const double expect = (double)a.n / vol * (4.0 / 3.0) * 3.141592653589793 * reach * reach * reach;
        const bool sd = a.tau != 0.0;  // spherodisks
        if (expect > 20.0) {
            if (sd) hipLaunchKernelGGL((k_migrate_platelet_wave<kPlateNearLong, true>), grid, block, 0, stream, a, L);
            else hipLaunchKernelGGL((k_migrate_platelet_wave<kPlateNearLong, false>), grid, block, 0, stream, a, L);
        } else {
            if (sd) hipLaunchKernelGGL((k_migrate_platelet_wave<kPlateNearShort, true>), grid, block, 0, stream, a, L);
            else hipLaunchKernelGGL((k_migrate_platelet_wave<kPlateNearShort, false>), grid, block, 0, stream, a, L);
        }
        main_done(SRM_KERNEL_PLATELET | SRM_KERNEL_WAVE);
    } else if (dim == 3) {
        if (poly) hipLaunchKernelGGL((k_migrate_wave<3, true>), grid, block, 0, stream, a, L);
        else hipLaunchKernelGGL((k_migrate_wave<3, false>), grid, block, 0, stream, a, L);
        main_done(SRM_KERNEL_WAVE);
    } else {
        if (poly) hipLaunchKernelGGL((k_migrate_wave<2, true>), grid, block, 0, stream, a, L);
        else hipLaunchKernelGGL((k_migrate_wave<2, false>), grid, block, 0, stream, a, L);
        main_done(SRM_KERNEL_WAVE);
    }
    return hipGetLastError();
}

hipError_t check_overlaps(int dim, int shape, bool poly, const PassArgs &a, bool check_all,
                          Counters *cnt, hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    if (shape != SRM_PLATELET && !check_all && wave_cells(dim, a.g, a.n)) {
        // crowded cells: one wavefront per failed particle
        const unsigned wb = blocks_for(a.n) < 1024 ? blocks_for(a.n) : 1024;
        if (dim == 3) {
            if (poly) hipLaunchKernelGGL((k_check_ball_wave<3, true>), dim3(wb), dim3(kBlock), 0, stream, a, cnt);
            else hipLaunchKernelGGL((k_check_ball_wave<3, false>), dim3(wb), dim3(kBlock), 0, stream, a, cnt);
        } else {
            if (poly) hipLaunchKernelGGL((k_check_ball_wave<2, true>), dim3(wb), dim3(kBlock), 0, stream, a, cnt);
            else hipLaunchKernelGGL((k_check_ball_wave<2, false>), dim3(wb), dim3(kBlock), 0, stream, a, cnt);
        }
        return hipGetLastError();
    }
    // grid-stride over the failed list (its length is only known on the device)
    const unsigned nb = blocks_for(a.n);
    const dim3 grid(check_all ? nb : (nb < 1024 ? nb : 1024)), block(kBlock);
    const int32_t all = check_all ? 1 : 0;
    if (shape == SRM_PLATELET) {
        if (a.tau != 0.0) hipLaunchKernelGGL(k_check_platelet<true>, grid, block, 0, stream, a, all, cnt);
        else hipLaunchKernelGGL(k_check_platelet<false>, grid, block, 0, stream, a, all, cnt);
    } else if (!check_all) {
        if (dim == 3) {
            if (poly) hipLaunchKernelGGL((k_check_ball_group<3, true>), grid, block, 0, stream, a, cnt);
            else hipLaunchKernelGGL((k_check_ball_group<3, false>), grid, block, 0, stream, a, cnt);
        } else {
            if (poly) hipLaunchKernelGGL((k_check_ball_group<2, true>), grid, block, 0, stream, a, cnt);
            else hipLaunchKernelGGL((k_check_ball_group<2, false>), grid, block, 0, stream, a, cnt);
        }
    } else if (dim == 3) {
        if (poly) hipLaunchKernelGGL((k_check_ball<3, true>), grid, block, 0, stream, a, all, cnt);
        else hipLaunchKernelGGL((k_check_ball<3, false>), grid, block, 0, stream, a, all, cnt);
    } else {
        if (poly) hipLaunchKernelGGL((k_check_ball<2, true>), grid, block, 0, stream, a, all, cnt);
        else hipLaunchKernelGGL((k_check_ball<2, false>), grid, block, 0, stream, a, all, cnt);
    }
    return hipGetLastError();
}

}  // namespace srm
