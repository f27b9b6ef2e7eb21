// Reference Philox4x32-10 taken from rocRAND's engine (an implementation
// independent of this repository), exported for the oracle's pin tests.
#include <rocrand/rocrand_philox4x32_10.h>
#include <stdint.h>

namespace {
struct Engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};
}  // namespace

extern "C" void ref_philox4x32(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n)
{
    Engine e;
    for (int64_t i = 0; i < n; ++i) {
        uint4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k = {key[2 * i], key[2 * i + 1]};
        uint4 r = e.ten_rounds(c, k);
        out[4 * i] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}
