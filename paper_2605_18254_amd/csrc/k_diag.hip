// k_diag.hip -- diagnostics of the device arithmetic the bit-exact contract
// rests on: IEEE binary64 sqrt and division as compiled for gfx950, the
// Philox4x32-10 generator, and the random-vector draw of a trial move.
#include "srm_internal.hpp"

namespace srm {
namespace {

__global__ void k_fp(const double *__restrict__ a, const double *__restrict__ b, int32_t n,
                     double *__restrict__ sq, double *__restrict__ dv)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sq[i] = __builtin_sqrt(a[i]);
    dv[i] = a[i] / b[i];
}

__global__ void k_philox(const uint32_t *__restrict__ ctr, const uint32_t *__restrict__ key,
                         int32_t n, uint32_t *__restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x0 = ctr[4 * i], x1 = ctr[4 * i + 1], x2 = ctr[4 * i + 2], x3 = ctr[4 * i + 3];
    philox4x32_10(x0, x1, x2, x3, key[2 * i], key[2 * i + 1]);
    out[4 * i] = x0;
    out[4 * i + 1] = x1;
    out[4 * i + 2] = x2;
    out[4 * i + 3] = x3;
}

__global__ void k_unitvec(int dim, Draw d, uint32_t stream, double len, int32_t n,
                          double *__restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[3];
    if (dim == 3) unit_vector<3>(d, (uint32_t)i, stream, len, v);
    else unit_vector<2>(d, (uint32_t)i, stream, len, v);
    out[3 * i] = v[0];
    out[3 * i + 1] = v[1];
    out[3 * i + 2] = v[2];
}

}  // namespace

hipError_t diag_fp(const double *a, const double *b, int32_t n, double *sq, double *dv,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_fp, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n, sq, dv);
    return hipGetLastError();
}

hipError_t diag_philox(const uint32_t *ctr, const uint32_t *key, int32_t n, uint32_t *out,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, s, ctr, key, n, out);
    return hipGetLastError();
}

hipError_t diag_unitvec(int dim, uint64_t seed, uint32_t t, uint32_t word, uint32_t stream,
                        double len, int32_t n, double *out, hipStream_t s)
{
    Draw d{(uint32_t)seed, (uint32_t)(seed >> 32), t, word};
    hipLaunchKernelGGL(k_unitvec, dim3((n + 255) / 256), dim3(256), 0, s, dim, d, stream, len, n,
                       out);
    return hipGetLastError();
}

}  // namespace srm
