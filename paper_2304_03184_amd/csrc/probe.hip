// Measurement probe: the rate of random 16-byte gathers this device sustains
// over a table of a given footprint, laid out and split across the XCDs the
// way the level-split hash-grid gather reads its table.  It is the practical
// ceiling the gather is compared against (its random loads are bound by the
// L1 -> L2 request rate long before HBM bandwidth); it plays no part in the
// method itself.
#include "common.hpp"

namespace nvr {
namespace {

// 32-bit integer finaliser (xorshift-multiply; constants from C. Wellons'
// published "lowbias32" search)
__device__ __forceinline__ uint32_t mix32(uint32_t v) {
    v ^= v >> 16;
    v *= 0x7feb352du;
    v ^= v >> 15;
    v *= 0x846ca68bu;
    v ^= v >> 16;
    return v;
}

// Workgroup b serves group b % 8, whose slice is the g-th eighth of the table.
// Item s of a group issues `loads` independent 16-byte loads at uniformly
// random aligned offsets of its slice, four at a time, and stores the xor of
// what it read (so no load can be dropped).
__global__ void __launch_bounds__(256)
probe_gather(const uint4 *__restrict__ table, uint32_t group_words, int64_t n, int loads,
             uint32_t seed, uint32_t *__restrict__ out) {
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const uint4 *slice = table + (size_t)g * group_words;
    for (int64_t c = blockIdx.x / kXcds; c * blockDim.x < n; c += chunks) {
        const int64_t s = c * blockDim.x + threadIdx.x;
        if (s >= n) break;
        const uint32_t h = mix32((uint32_t)s ^ mix32(seed + (uint32_t)g));
        uint32_t acc = 0u;
        for (int j = 0; j < loads; j += 4) {
            uint4 q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t r = mix32(h + (uint32_t)(j + k) * 0x9e3779b9u);
                q[k] = slice[((uint64_t)r * group_words) >> 32];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) acc ^= q[k].x ^ q[k].y ^ q[k].z ^ q[k].w;
        }
        out[(size_t)g * n + s] = acc;
    }
}

}  // namespace
}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_probe_gather(const void *table, size_t bytes, int64_t n, int32_t loads,
                                       uint32_t seed, uint32_t *out, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(n >= 0 && n < (1ll << 31), NVR_EINVAL, "n out of range");
    NVR_REQUIRE(loads > 0 && loads % 4 == 0 && loads <= 1024, NVR_EINVAL,
                "loads must be a positive multiple of 4, at most 1024");
    const size_t group_words = bytes / 16 / kXcds;
    NVR_REQUIRE(group_words >= 1 && group_words < (1ull << 32), NVR_EINVAL,
                "table must hold 8 .. 2^35 16-byte words");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(table && out, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(table, 16) && aligned(out, 4), NVR_EINVAL, "misaligned array");
    const unsigned grid = grid_for(n, 256, 2048) * kXcds;
    probe_gather<<<grid, 256, 0, hs(stream)>>>((const uint4 *)table, (uint32_t)group_words, n,
                                               loads, seed, out);
    NVR_LAUNCHED();
    return NVR_OK;
}
