// Shared host/device helpers of the nvr library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdarg.h>
#include <string>

#include "nvr.h"

namespace nvr {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

#define NVR_REQUIRE(cond, code, ...)                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            ::nvr::set_error(__VA_ARGS__);                             \
            return (code);                                             \
        }                                                              \
    } while (0)

#define NVR_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            ::nvr::set_error("%s failed: %s (%s:%d)", #call,                   \
                             hipGetErrorString(e_), __FILE__, __LINE__);       \
            return NVR_EHIP;                                                   \
        }                                                                      \
    } while (0)

#define NVR_LAUNCHED()                                                         \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) {                                                \
            ::nvr::set_error("kernel launch failed: %s (%s:%d)",               \
                             hipGetErrorString(e_), __FILE__, __LINE__);       \
            return NVR_EHIP;                                                   \
        }                                                                      \
    } while (0)

#define NVR_TRY(expr)                                                          \
    do {                                                                       \
        nvr_status s_ = (expr);                                                \
        if (s_ != NVR_OK) return s_;                                           \
    } while (0)

inline hipStream_t hs(nvr_stream s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned(const void *p, size_t a) {
    return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

// Grid size for a grid-stride launch over `n` items with `block` threads,
// capped at `cap` blocks (a multiple of the 8 XCDs).
inline unsigned grid_for(int64_t n, int block, int64_t cap = 8192) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

constexpr int kXcds = 8;          // MI355X: 8 XCDs, 32 CUs each
constexpr int kCus = 256;

// ---------------------------------------------------------------- device
__device__ __forceinline__ int64_t count_of(int64_t n, const int32_t *n_dev, int64_t cap) {
    if (n_dev == nullptr) return n;
    int64_t v = *n_dev;
    return v < cap ? v : cap;
}

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;      // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                          // round to nearest even
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_bits(float f) {
    _Float16 h = static_cast<_Float16>(f);
    return *reinterpret_cast<uint16_t *>(&h);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
    _Float16 h = *reinterpret_cast<_Float16 *>(&b);
    return static_cast<float>(h);
}

}  // namespace nvr
