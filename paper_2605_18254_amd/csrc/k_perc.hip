// k_perc.hip -- hard core-soft shell percolation of a committed
// configuration (the critical percolation distance of the paper's
// Sec. 3.3): particles are bonded when they overlap after growing by the
// gap (the srm_pairs predicate), and a cluster percolates along axis a when
// it wraps around the periodic box along a, i.e. some cycle of bonds has a
// nonzero winding along a.
//
// Every particle carries (label, offset): the smallest id found so far in
// its cluster and its periodic image (integer box shifts per axis) relative
// to that particle.  A bond i -> j with image shift s (j's image nearest i
// is x_j + s L) offers j the state (label_i, offset_i + s) and i the state
// (label_j, offset_j - s); a particle takes an offer only when its label is
// strictly smaller, by compare-and-swap, so each (particle, label) state is
// written once.  When nothing changes, every cluster carries its smallest id
// and offsets taken along a spanning tree of bonds; a bond whose offsets
// disagree (offset_i + s != offset_j) closes a cycle with that winding, and
// the cycles through non-tree bonds generate all the cluster's cycles, so
// the axes where some bond disagrees are exactly the percolating axes.
#include "srm_internal.hpp"

namespace srm {
namespace {

constexpr int kBlock = 256;
constexpr int kOffBits = 10;  // per axis, biased
constexpr int32_t kOffBias = 1 << (kOffBits - 1);

inline unsigned blocks_for(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b > 0 ? (b < 65535 * 16 ? b : 65535 * 16) : 1);
}

__device__ __forceinline__ unsigned long long pack(int32_t label, const int32_t off[3])
{
    unsigned long long o = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) o |= (unsigned long long)(uint32_t)(off[a] + kOffBias) << (kOffBits * a);
    return ((unsigned long long)(uint32_t)label << 32) | o;
}

__device__ __forceinline__ int32_t label_of(unsigned long long v) { return (int32_t)(v >> 32); }

__device__ __forceinline__ void offsets_of(unsigned long long v, int32_t off[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        off[a] = (int32_t)((v >> (kOffBits * a)) & ((1u << kOffBits) - 1u)) - kOffBias;
}

// Image shift of bond (i, j): s_a = +1 when x_j - x_i < -L/2 (j's nearest
// image is x_j + L), -1 when x_j - x_i > L/2, else 0.  Packed 8 bits per axis.
__global__ void __launch_bounds__(kBlock) k_bond_shift(const int32_t *__restrict__ ij, int64_t nb,
                                                       const double *__restrict__ pos, int32_t n,
                                                       int dim, Grid g,
                                                       int32_t *__restrict__ shift)
{
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = ij[2 * b], j = ij[2 * b + 1];
        int32_t packed = 0;
        for (int a = 0; a < dim; ++a) {
            const double d = pos[(size_t)a * n + j] - pos[(size_t)a * n + i];
            const int32_t s = (d > g.half[a]) ? -1 : ((d < -g.half[a]) ? 1 : 0);
            packed |= (s & 0xff) << (8 * a);
        }
        shift[b] = packed;
    }
}

__device__ __forceinline__ void unpack_shift(int32_t packed, int32_t s[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = (int32_t)(int8_t)((packed >> (8 * a)) & 0xff);
}

__global__ void __launch_bounds__(kBlock) k_perc_init(unsigned long long *__restrict__ state,
                                                      int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t zero[3] = {0, 0, 0};
    state[i] = pack(i, zero);
}

// Offer `v` to node k: taken only if its label is strictly smaller.
__device__ __forceinline__ bool offer(unsigned long long *state, int32_t k, unsigned long long v)
{
    unsigned long long cur = state[k];
    while (label_of(v) < label_of(cur)) {
        const unsigned long long prev = atomicCAS(&state[k], cur, v);
        if (prev == cur) return true;
        cur = prev;
    }
    return false;
}

__global__ void __launch_bounds__(kBlock) k_perc_relax(const int32_t *__restrict__ ij,
                                                       const int32_t *__restrict__ shift, int64_t nb,
                                                       unsigned long long *state,
                                                       int32_t *__restrict__ flags)
{
    bool changed = false, overflow = false;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = ij[2 * b], j = ij[2 * b + 1];
        int32_t s[3];
        unpack_shift(shift[b], s);
        const unsigned long long si = __atomic_load_n(&state[i], __ATOMIC_RELAXED);
        const unsigned long long sj = __atomic_load_n(&state[j], __ATOMIC_RELAXED);
        const int32_t li = label_of(si), lj = label_of(sj);
        if (li == lj) continue;
        int32_t o[3];
        if (li < lj) {
            offsets_of(si, o);
            for (int a = 0; a < 3; ++a) {
                o[a] += s[a];
                overflow = overflow || o[a] <= -kOffBias || o[a] >= kOffBias - 1;
            }
            changed = offer(state, j, pack(li, o)) || changed;
        } else {
            offsets_of(sj, o);
            for (int a = 0; a < 3; ++a) {
                o[a] -= s[a];
                overflow = overflow || o[a] <= -kOffBias || o[a] >= kOffBias - 1;
            }
            changed = offer(state, i, pack(lj, o)) || changed;
        }
    }
    if (changed) atomicOr(&flags[0], 1);
    if (overflow) atomicOr(&flags[1], 1);
}

// After convergence: the axes along which some bond's offsets disagree.
__global__ void __launch_bounds__(kBlock) k_perc_check(const int32_t *__restrict__ ij,
                                                       const int32_t *__restrict__ shift, int64_t nb,
                                                       const unsigned long long *__restrict__ state,
                                                       int32_t *__restrict__ flags)
{
    int32_t mask = 0;
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = ij[2 * b], j = ij[2 * b + 1];
        int32_t s[3], oi[3], oj[3];
        unpack_shift(shift[b], s);
        offsets_of(state[i], oi);
        offsets_of(state[j], oj);
        for (int a = 0; a < 3; ++a)
            if (oi[a] + s[a] != oj[a]) mask |= 1 << a;
    }
    if (mask) atomicOr(&flags[2], mask);
}

}  // namespace

hipError_t bond_shifts(const int32_t *ij, int64_t nb, const double *pos_by_id, int32_t n, int dim,
                       const Grid &g, int32_t *shift, hipStream_t stream)
{
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bond_shift, dim3(blocks_for(nb)), dim3(kBlock), 0, stream, ij, nb,
                       pos_by_id, n, dim, g, shift);
    return hipGetLastError();
}

hipError_t perc_init(unsigned long long *state, int32_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_perc_init, dim3(blocks_for(n)), dim3(kBlock), 0, stream, state, n);
    return hipGetLastError();
}

hipError_t perc_relax(const int32_t *ij, const int32_t *shift, int64_t nb,
                      unsigned long long *state, int32_t *flags, hipStream_t stream)
{
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_perc_relax, dim3(blocks_for(nb)), dim3(kBlock), 0, stream, ij, shift, nb,
                       state, flags);
    return hipGetLastError();
}

hipError_t perc_check(const int32_t *ij, const int32_t *shift, int64_t nb,
                      const unsigned long long *state, int32_t *flags, hipStream_t stream)
{
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_perc_check, dim3(blocks_for(nb)), dim3(kBlock), 0, stream, ij, shift, nb,
                       state, flags);
    return hipGetLastError();
}

}  // namespace srm
