// Ray clipping and occupancy-skipping sample placement.
//
// Three launches, no host synchronisation:
//   1. march_count  -- one thread per ray: clip, walk the steps, count kept
//                      samples; 256-ray block scan in LDS -> local offsets,
//                      block totals;
//   2. scan_blocks  -- one workgroup scans the block totals, writes the total
//                      sample count to n_dev and off[R];
//   3. march_write  -- a group of 16 lanes per ray walks again, 16 steps at a
//                      time, and writes t, dt, x and the ray id of the kept
//                      samples at the ray's global offset (capacity-bounded);
//                      the kept samples of a 16-step chunk are numbered by a
//                      group ballot, so they are stored as one contiguous run.
// The walk's integer decisions use IEEE float32 with one rounding per
// operation (floating-point contraction is switched off in those functions,
// so no multiply-add is fused), in the order fixed by the documented reading.
#include "common.hpp"

#include <cmath>
#include <mutex>

namespace nvr {

struct MarchParams {
    float lo[3], hi[3];
    float near_t, far_t, step;
    float occ_scale[3];
    int max_steps, occ_res;
    int64_t begin, end;
};

struct RaySeg {
    float tn, tf;
};

__device__ __forceinline__ RaySeg clip_ray(const MarchParams &p, const float *o, const float *d) {
#pragma clang fp contract(off)
    float tn = p.near_t, tf = p.far_t;
    float lo_t[3], hi_t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float inv = 1.0f / d[a];
        const float t0 = (p.lo[a] - o[a]) * inv;
        const float t1 = (p.hi[a] - o[a]) * inv;
        lo_t[a] = fminf(t0, t1);
        hi_t[a] = fmaxf(t0, t1);
    }
    tn = fmaxf(fmaxf(fmaxf(lo_t[0], lo_t[1]), lo_t[2]), tn);
    tf = fminf(fminf(fminf(hi_t[0], hi_t[1]), hi_t[2]), tf);
    return {tn, tf};
}

__device__ __forceinline__ bool occupied(const MarchParams &p, const uint32_t *occ,
                                         const float x[3]) {
#pragma clang fp contract(off)
    if (p.occ_res == 0) return true;
    int v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = (x[a] - p.lo[a]) * p.occ_scale[a];
        int c = (int)floorf(u);
        c = c < 0 ? 0 : (c > p.occ_res - 1 ? p.occ_res - 1 : c);
        v[a] = c;
    }
    const uint32_t idx = (uint32_t)v[0] + (uint32_t)p.occ_res * ((uint32_t)v[1] +
                                                                (uint32_t)p.occ_res * (uint32_t)v[2]);
    return (occ[idx >> 5] >> (idx & 31u)) & 1u;
}

// Walks ray r; calls emit(i_kept, t, x) for every kept sample; returns the count.
template <typename Emit>
__device__ __forceinline__ int walk(const MarchParams &p, const uint32_t *occ, const float *o,
                                    const float *d, Emit emit) {
#pragma clang fp contract(off)
    const RaySeg s = clip_ray(p, o, d);
    int kept = 0;
    if (!(s.tf > s.tn)) return 0;
    for (int i = 0; i < p.max_steps; ++i) {
        const float t = s.tn + ((float)i + 0.5f) * p.step;
        if (!(t < s.tf)) break;
        float x[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
        if (occupied(p, occ, x)) {
            emit(kept, t, x);
            ++kept;
        }
    }
    return kept;
}

constexpr int kMarchBlock = 256;

__global__ void __launch_bounds__(kMarchBlock)
march_count(MarchParams p, int64_t n_rays, const float *__restrict__ o,
            const float *__restrict__ d, const uint32_t *__restrict__ occ,
            int32_t *__restrict__ off, int32_t *__restrict__ block_sums) {
    __shared__ int32_t buf[kMarchBlock];
    const int64_t r = blockIdx.x * (int64_t)kMarchBlock + threadIdx.x;
    int cnt = 0;
    if (r < n_rays && r >= p.begin && r < p.end) {
        float oo[3] = {o[3 * r], o[3 * r + 1], o[3 * r + 2]};
        float dd[3] = {d[3 * r], d[3 * r + 1], d[3 * r + 2]};
        cnt = walk(p, occ, oo, dd, [](int, float, const float *) {});
    }
    // inclusive Hillis-Steele scan in LDS
    buf[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = 1; s < kMarchBlock; s <<= 1) {
        int v = threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
        __syncthreads();
        buf[threadIdx.x] += v;
        __syncthreads();
    }
    if (r < n_rays) off[r] = buf[threadIdx.x] - cnt;   // exclusive, block-local
    if (threadIdx.x == kMarchBlock - 1) block_sums[blockIdx.x] = buf[kMarchBlock - 1];
}

// Single workgroup: exclusive scan of nb block sums in place; total -> n_dev, off[n_rays].
__global__ void __launch_bounds__(1024)
scan_blocks(int64_t nb, int32_t *__restrict__ block_sums, int64_t n_rays, int64_t capacity,
            int32_t *__restrict__ off, int32_t *__restrict__ n_dev) {
    __shared__ int32_t buf[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < nb ? block_sums[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < 1024; s <<= 1) {
            int32_t u = threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
            __syncthreads();
            buf[threadIdx.x] += u;
            __syncthreads();
        }
        if (i < nb) block_sums[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // offsets are clamped to the capacity so that no consumer reads past the
        // sample arrays; n_dev keeps the true total (overflow detection)
        off[n_rays] = carry < capacity ? carry : (int32_t)capacity;
        *n_dev = carry;
    }
}

constexpr int kRayGroup = 16;   // lanes per ray in march_write

__global__ void __launch_bounds__(kMarchBlock)
march_write(MarchParams p, int64_t n_rays, const float *__restrict__ o,
            const float *__restrict__ d, const uint32_t *__restrict__ occ,
            const int32_t *__restrict__ block_sums, int64_t capacity, int32_t *__restrict__ off,
            int32_t *__restrict__ ray_id, float *__restrict__ t_out, float *__restrict__ dt_out,
            float *__restrict__ x_out) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x % kRayGroup;
    const int64_t r = (blockIdx.x * (int64_t)kMarchBlock + threadIdx.x) / kRayGroup;
    if (r >= n_rays) return;                       // the same for the whole group
    // every lane of the group reads off[r] before lane 0 rewrites it (one
    // wavefront, program order)
    const int64_t base = (int64_t)off[r] + block_sums[r / kMarchBlock];
    if (lane == 0) off[r] = (int32_t)(base < capacity ? base : capacity);
    if (r < p.begin || r >= p.end) return;
    const float oo[3] = {o[3 * r], o[3 * r + 1], o[3 * r + 2]};
    const float dd[3] = {d[3 * r], d[3 * r + 1], d[3 * r + 2]};
    const RaySeg sg = clip_ray(p, oo, dd);
    if (!(sg.tf > sg.tn)) return;
    const int first = (threadIdx.x % 64) & ~(kRayGroup - 1);   // group's first lane in the wave
    int64_t kept = 0;
    for (int i0 = 0; i0 < p.max_steps; i0 += kRayGroup) {
        // step i = i0 + lane, with the same arithmetic as the sequential walk
        const int i = i0 + lane;
        bool live = false, keep = false;
        float t = 0.f, x[3] = {0.f, 0.f, 0.f};
        if (i < p.max_steps) {
            t = sg.tn + ((float)i + 0.5f) * p.step;
            if (t < sg.tf) {
                live = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) x[a] = oo[a] + t * dd[a];
                keep = occupied(p, occ, x);
            }
        }
        const uint32_t gk = (uint32_t)(__ballot(keep) >> first) & 0xffffu;
        const uint32_t gl = (uint32_t)(__ballot(live) >> first) & 0xffffu;
        if (keep) {
            const int64_t j = base + kept + __popc(gk & ((1u << lane) - 1u));
            if (j < capacity) {
                ray_id[j] = (int32_t)r;
                t_out[j] = t;
                dt_out[j] = p.step;
                x_out[3 * j] = x[0];
                x_out[3 * j + 1] = x[1];
                x_out[3 * j + 2] = x[2];
            }
        }
        kept += __popc(gk);
        if (gl != 0xffffu) break;                  // the walk ended inside this chunk
    }
}

nvr_status make_march_params(const nvr_march_desc *m, int64_t begin, int64_t end,
                             MarchParams *p) {
    NVR_REQUIRE(m != nullptr, NVR_EINVAL, "march descriptor is NULL");
    NVR_REQUIRE(m->max_steps >= 1 && m->max_steps <= 1024, NVR_EINVAL, "max_steps out of 1..1024");
    NVR_REQUIRE(m->occ_res >= 0 && m->occ_res <= 1024, NVR_EINVAL, "occ_res out of 0..1024");
    double side_max = 0.0;
    for (int a = 0; a < 3; ++a) {
        NVR_REQUIRE(m->aabb_max[a] > m->aabb_min[a], NVR_EINVAL, "empty box on axis %d", a);
        const double side = (double)m->aabb_max[a] - (double)m->aabb_min[a];
        side_max = side > side_max ? side : side_max;
        p->lo[a] = m->aabb_min[a];
        p->hi[a] = m->aabb_max[a];
        p->occ_scale[a] = m->occ_res > 0 ? (float)((double)m->occ_res / side) : 0.f;
    }
    p->near_t = m->near_t;
    p->far_t = m->far_t;
    p->step = m->step > 0.f ? m->step : (float)(std::sqrt(3.0) * side_max / (double)m->max_steps);
    p->max_steps = m->max_steps;
    p->occ_res = m->occ_res;
    p->begin = begin;
    p->end = end;
    return NVR_OK;
}

int64_t march_blocks(int64_t n_rays) { return (n_rays + kMarchBlock - 1) / kMarchBlock; }

nvr_status launch_march(const MarchParams &p, int64_t n_rays, const float *o, const float *d,
                        const uint32_t *occ, int64_t capacity, int32_t *off, int32_t *ray_id,
                        float *t, float *dt, float *x, int32_t *n_dev, int32_t *block_sums,
                        hipStream_t st) {
    const int64_t nb = march_blocks(n_rays);
    if (nb > 0) {
        march_count<<<(unsigned)nb, kMarchBlock, 0, st>>>(p, n_rays, o, d, occ, off, block_sums);
        NVR_LAUNCHED();
    }
    scan_blocks<<<1, 1024, 0, st>>>(nb, block_sums, n_rays, capacity, off, n_dev);
    NVR_LAUNCHED();
    if (nb > 0) {
        const int64_t nw = (n_rays * kRayGroup + kMarchBlock - 1) / kMarchBlock;
        march_write<<<(unsigned)nw, kMarchBlock, 0, st>>>(p, n_rays, o, d, occ, block_sums,
                                                          capacity, off, ray_id, t, dt, x);
        NVR_LAUNCHED();
    }
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" size_t nvr_march_workspace(int64_t n_rays) {
    if (n_rays < 0) return 0;
    return sizeof(int32_t) * (size_t)(march_blocks(n_rays) + 1);
}

extern "C" nvr_status nvr_march(const nvr_march_desc *m, int64_t n_rays, int64_t ray_begin,
                                int64_t ray_end, const float *o, const float *d,
                                const uint32_t *occ, int64_t capacity, int32_t *off,
                                int32_t *ray_id, float *t, float *dt, float *x, int32_t *n_dev,
                                void *workspace, nvr_stream stream) {
    clear_error();
    MarchParams p;
    NVR_TRY(make_march_params(m, ray_begin, ray_end, &p));
    NVR_REQUIRE(n_rays >= 0 && n_rays < (1ll << 31), NVR_EINVAL, "n_rays out of range");
    NVR_REQUIRE(ray_begin >= 0 && ray_begin <= ray_end && ray_end <= n_rays, NVR_EINVAL,
                "ray range [%lld, %lld) not inside [0, %lld)", (long long)ray_begin,
                (long long)ray_end, (long long)n_rays);
    NVR_REQUIRE(capacity >= 0 && capacity < (1ll << 31), NVR_EINVAL, "capacity out of range");
    NVR_REQUIRE(off && n_dev && workspace, NVR_EINVAL, "NULL off / n_dev / workspace");
    NVR_REQUIRE(m->occ_res == 0 || occ != nullptr, NVR_EINVAL, "occ is NULL but occ_res > 0");
    if (n_rays > 0) NVR_REQUIRE(o && d, NVR_EINVAL, "NULL rays");
    if (capacity > 0) NVR_REQUIRE(ray_id && t && dt && x, NVR_EINVAL, "NULL sample arrays");
    return launch_march(p, n_rays, o, d, occ, capacity, off, ray_id, t, dt, x, n_dev,
                        (int32_t *)workspace, hs(stream));
}

// ---------------------------------------------------------------- no-alloc entry
// nvr_march_noalloc keeps the per-block sums of the scan in a file-scope device
// array instead of a caller workspace.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): the device
// address is looked up once per device with hipGetSymbolAddress and kept.
namespace nvr {

constexpr int64_t kNoAllocMaxRays = 1ll << 24;
constexpr int kMaxDevices = 64;

}  // namespace nvr

static __device__ __align__(256) int32_t scratch[nvr::kNoAllocMaxRays / nvr::kMarchBlock + 1];

namespace nvr {

static std::mutex g_scratch_mu;
static int32_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
static nvr_status scratch_on_current_device(hipStream_t st, int32_t **out) {
    int dev = -1;
    NVR_HIP(hipGetDevice(&dev));
    NVR_REQUIRE(dev >= 0 && dev < kMaxDevices, NVR_EUNSUPPORTED, "device %d beyond %d", dev,
                kMaxDevices);
    if (st != nullptr) {
        int sdev = -1;
        NVR_HIP(hipStreamGetDevice(st, &sdev));
        NVR_REQUIRE(sdev == dev, NVR_EINVAL,
                    "stream belongs to device %d but device %d is current", sdev, dev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        NVR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        NVR_REQUIRE(p != nullptr, NVR_EHIP, "hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = static_cast<int32_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return NVR_OK;
}

}  // namespace nvr

extern "C" nvr_status nvr_march_noalloc(const nvr_march_desc *m, int64_t n_rays,
                                        int64_t ray_begin, int64_t ray_end, const float *o,
                                        const float *d, const uint32_t *occ, int64_t capacity,
                                        int32_t *off, int32_t *ray_id, float *t, float *dt,
                                        float *x, int32_t *n_dev, nvr_stream stream) {
    clear_error();
    MarchParams p;
    NVR_TRY(make_march_params(m, ray_begin, ray_end, &p));
    NVR_REQUIRE(n_rays >= 0 && n_rays <= kNoAllocMaxRays, NVR_EINVAL,
                "n_rays %lld outside 0..%lld (the fixed scratch holds the block sums of at "
                "most 2^24 rays)", (long long)n_rays, (long long)kNoAllocMaxRays);
    NVR_REQUIRE(ray_begin >= 0 && ray_begin <= ray_end && ray_end <= n_rays, NVR_EINVAL,
                "ray range [%lld, %lld) not inside [0, %lld)", (long long)ray_begin,
                (long long)ray_end, (long long)n_rays);
    NVR_REQUIRE(capacity >= 0 && capacity < (1ll << 31), NVR_EINVAL, "capacity out of range");
    NVR_REQUIRE(off && n_dev, NVR_EINVAL, "NULL off / n_dev");
    NVR_REQUIRE(m->occ_res == 0 || occ != nullptr, NVR_EINVAL, "occ is NULL but occ_res > 0");
    if (n_rays > 0) NVR_REQUIRE(o && d, NVR_EINVAL, "NULL rays");
    if (capacity > 0) NVR_REQUIRE(ray_id && t && dt && x, NVR_EINVAL, "NULL sample arrays");
    int32_t *ws = nullptr;
    NVR_TRY(scratch_on_current_device(hs(stream), &ws));
    // every block sum the scan reads is written by the count launch of this call
    return launch_march(p, n_rays, o, d, occ, capacity, off, ray_id, t, dt, x, n_dev, ws,
                        hs(stream));
}

#include "launch.hpp"

namespace nvr {

size_t march_ws_bytes(int64_t n_rays) { return nvr_march_workspace(n_rays); }

nvr_status march_desc_check(const nvr_march_desc *m) {
    MarchParams p;
    return make_march_params(m, 0, 0, &p);
}

nvr_status run_march(const nvr_march_desc *m, int64_t n_rays, int64_t begin, int64_t end,
                     const float *o, const float *d, const uint32_t *occ, int64_t capacity,
                     int32_t *off, int32_t *ray_id, float *t, float *dt, float *x, int32_t *n_dev,
                     int32_t *ws, hipStream_t st) {
    MarchParams p;
    NVR_TRY(make_march_params(m, begin, end, &p));
    return launch_march(p, n_rays, o, d, occ, capacity, off, ray_id, t, dt, x, n_dev, ws, st);
}

}  // namespace nvr
