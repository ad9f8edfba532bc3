// Binned backward of the hash encoding (table-gradient scatter without global
// float atomics per contribution).
//
// fp32 global atomics run at ~20 G/s on the whole device and serialise on the
// few entries of the coarse dense levels, which every sample hits; one step
// makes ~1.7 G of them.  Instead the scatter becomes a bucketed reduction:
//
//   count   every (sample, level, corner) contribution is assigned to the
//           16384-entry table tile holding its entry; per-workgroup LDS
//           histograms are added into per-tile counts;
//   scan    one workgroup turns the counts into tile ranges, resets the append
//           cursors and splits every tile into work items of <= 2^21 records
//           (a hashed-level tile is one item; the coarse dense tiles, which
//           every sample hits, are split);
//   emit    the contributions (entry, w * dfeat_0, w * dfeat_1) are recomputed
//           and appended to their tile's range: ranks come from LDS counters,
//           one global atomic per (workgroup chunk, tile) reserves the space;
//           the position gradient (for the warp) is formed here as well;
//   accum   each work item sums its records into an LDS copy of the tile
//           (ds_add_f32); a tile that is a single item is added into the
//           gradient table directly (plain read-modify-write, it owns the tile),
//           the items of a split tile write their sums to partial slabs which
//           a last launch adds up per entry -- no global atomics at all.
//
// Levels are split over the XCDs as in the forward (workgroup b serves level
// group b % 8) in count and emit.
#include "common.hpp"
#include "grid_dev.hpp"
#include "scatter_dev.hpp"

namespace nvr {

constexpr int kTileBits = 14;
constexpr int kTileEntries = 1 << kTileBits;
constexpr uint32_t kItemRecords = 1u << 21;
constexpr int kBinBlock = 256;
constexpr int kAccumBlock = 1024;
constexpr int kMaxLpg = 4;   // levels per group (L <= 32)

static int64_t max_items_of(int64_t cap, int L, int nt) {
    return (int64_t)cap * L * 8 / kItemRecords + nt + 1;
}

int scatter_tiles(const GridParams &p) {
    return (int)(((int64_t)p.off[p.L] + kTileEntries - 1) >> kTileBits);
}

size_t scatter_ws_bytes(const GridParams &p, int64_t cap) {
    const int nt = scatter_tiles(p);
    const size_t max_rec = (size_t)cap * p.L * 8;
    size_t b = 0;
    b += sizeof(uint32_t) * (size_t)(4 * (nt + 1) + 4);  // counts, starts, cursors, items, n
    b = (b + 255) & ~size_t(255);
    b += sizeof(uint32_t) * max_rec;                     // keys
    b = (b + 255) & ~size_t(255);
    b += sizeof(float2) * max_rec;                       // values
    b = (b + 255) & ~size_t(255);
    b += sizeof(float) * 2 * kTileEntries * (size_t)max_items_of(cap, p.L, nt);  // partial slabs
    return b;
}

struct ScatterWs {
    uint32_t *count, *start, *cursor, *item_start, *n_items;
    uint32_t *keys;
    float2 *vals;
    float *partial;       // [max_items][2 * kTileEntries]
};

static ScatterWs carve_scatter(const GridParams &p, void *ws, int64_t cap) {
    const int nt = scatter_tiles(p);
    const size_t max_rec = (size_t)cap * p.L * 8;
    ScatterWs w;
    uint32_t *u = (uint32_t *)ws;
    w.count = u;
    w.start = u + (nt + 1);
    w.cursor = u + 2 * (nt + 1);
    w.item_start = u + 3 * (nt + 1);
    w.n_items = u + 4 * (nt + 1);
    size_t b = sizeof(uint32_t) * (size_t)(4 * (nt + 1) + 4);
    b = (b + 255) & ~size_t(255);
    w.keys = (uint32_t *)((char *)ws + b);
    b += sizeof(uint32_t) * max_rec;
    b = (b + 255) & ~size_t(255);
    w.vals = (float2 *)((char *)ws + b);
    b += sizeof(float2) * max_rec;
    b = (b + 255) & ~size_t(255);
    w.partial = (float *)((char *)ws + b);
    return w;
}

__global__ void zero_u32(uint32_t *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- count
__global__ void __launch_bounds__(kBinBlock)
scatter_count(GridParams p, int n_tiles, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
              const float *__restrict__ x, uint32_t *__restrict__ tile_count) {
    extern __shared__ uint32_t hist[];
    for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) hist[t] = 0u;
    __syncthreads();
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int lpg = (p.L + kXcds - 1) / kXcds;
    for (int64_t c = blockIdx.x / kXcds; c * blockDim.x < count; c += chunks) {
        const int64_t s = c * blockDim.x + threadIdx.x;
        if (s < count) {
            const float px = x[3 * s], py = x[3 * s + 1], pz = x[3 * s + 2];
            for (int m = 0; m < lpg; ++m) {
                const int l = g + kXcds * m;
                if (l >= p.L) break;
                const LevelPos lp = level_pos(p, l, px, py, pz);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t e = p.off[l] + corner_index(p, l, lp, k);
                    atomicAdd(&hist[e >> kTileBits], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n_tiles; t += blockDim.x)
        if (hist[t]) atomicAdd(&tile_count[t], hist[t]);
}

// ---------------------------------------------------------------- scan
__global__ void __launch_bounds__(1024)
scatter_scan(int n_tiles, const uint32_t *__restrict__ tile_count, uint32_t *__restrict__ start,
             uint32_t *__restrict__ cursor, uint32_t *__restrict__ item_start,
             uint32_t *__restrict__ n_items) {
    __shared__ uint32_t a[1024], b[1024];
    __shared__ uint32_t carry_r, carry_i;
    if (threadIdx.x == 0) {
        carry_r = 0;
        carry_i = 0;
    }
    __syncthreads();
    for (int base = 0; base < n_tiles; base += 1024) {
        const int t = base + threadIdx.x;
        const uint32_t c = t < n_tiles ? tile_count[t] : 0u;
        const uint32_t it = (c + kItemRecords - 1) / kItemRecords;
        a[threadIdx.x] = c;
        b[threadIdx.x] = it;
        __syncthreads();
        for (int s = 1; s < 1024; s <<= 1) {
            const uint32_t va = threadIdx.x >= s ? a[threadIdx.x - s] : 0u;
            const uint32_t vb = threadIdx.x >= s ? b[threadIdx.x - s] : 0u;
            __syncthreads();
            a[threadIdx.x] += va;
            b[threadIdx.x] += vb;
            __syncthreads();
        }
        if (t < n_tiles) {
            const uint32_t sr = carry_r + a[threadIdx.x] - c;
            start[t] = sr;
            cursor[t] = sr;
            item_start[t] = carry_i + b[threadIdx.x] - it;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry_r += a[1023];
            carry_i += b[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        start[n_tiles] = carry_r;
        item_start[n_tiles] = carry_i;
        *n_items = carry_i;
    }
}

// ---------------------------------------------------------------- emit
template <bool PLANAR, int LPG>
__global__ void __launch_bounds__(kBinBlock)
scatter_emit(GridParams p, int n_tiles, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
             const float *__restrict__ x, const uint32_t *__restrict__ table,
             const float *__restrict__ dfeat, const uint32_t *__restrict__ start,
             uint32_t *__restrict__ cursor, uint32_t *__restrict__ keys, float2 *__restrict__ vals,
             float *__restrict__ dx_parts) {
    extern __shared__ uint32_t lds[];
    uint32_t *hist = lds;                 // [n_tiles] ranks
    uint32_t *base = lds + n_tiles;       // [n_tiles] reserved positions
    uint32_t *end = lds + 2 * n_tiles;    // [n_tiles] end of each tile's range
    for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) end[t] = start[t + 1];
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int lpg = LPG;
    for (int64_t c = blockIdx.x / kXcds; c * blockDim.x < count; c += chunks) {
        for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) hist[t] = 0u;
        __syncthreads();
        const int64_t s = c * blockDim.x + threadIdx.x;
        const bool valid = s < count;
        uint32_t ent[LPG * 8], rank[LPG * 8];
        float v0[LPG * 8], v1[LPG * 8];
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;
        float px = 0.f, py = 0.f, pz = 0.f;
        if (valid) {
            px = x[3 * s];
            py = x[3 * s + 1];
            pz = x[3 * s + 2];
        }
#pragma unroll
        for (int m = 0; m < LPG; ++m) {
            const int l = g + kXcds * m;
            const bool on = valid && l < p.L;
            float g0 = 0.f, g1 = 0.f;
            LevelPos lp;
            if (on) {
                lp = level_pos(p, l, px, py, pz);
                if (PLANAR) {
                    const float *src = dfeat + ((size_t)g * cap + s) * (2 * lpg) + 2 * m;
                    g0 = src[0];
                    g1 = src[1];
                } else {
                    g0 = dfeat[(size_t)s * (2 * p.L) + 2 * l];
                    g1 = dfeat[(size_t)s * (2 * p.L) + 2 * l + 1];
                }
            }
            float e0 = 0.f, e1 = 0.f, e2 = 0.f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int r = 8 * m + k;
                if (on) {
                    const float w = corner_weight(lp, k);
                    const uint32_t e = p.off[l] + corner_index(p, l, lp, k);
                    ent[r] = e;
                    v0[r] = w * g0;
                    v1[r] = w * g1;
                    rank[r] = atomicAdd(&hist[e >> kTileBits], 1u);
                    if (dx_parts != nullptr) {
                        const uint32_t v = table[e];
                        const float tg = f16_bits_to_f32((uint16_t)(v & 0xffffu)) * g0 +
                                         f16_bits_to_f32((uint16_t)(v >> 16)) * g1;
                        const float3 dw = corner_dweight(lp, k);
                        e0 += dw.x * tg;
                        e1 += dw.y * tg;
                        e2 += dw.z * tg;
                    }
                } else {
                    ent[r] = 0xffffffffu;
                }
            }
            if (on && dx_parts != nullptr) {
                const float N = (float)p.res[l];
                if (lp.inside[0]) d0 += e0 * N * (float)p.inv_side[0];
                if (lp.inside[1]) d1 += e1 * N * (float)p.inv_side[1];
                if (lp.inside[2]) d2 += e2 * N * (float)p.inv_side[2];
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) {
            const uint32_t h = hist[t];
            base[t] = h ? atomicAdd(&cursor[t], h) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < LPG * 8; ++r) {
            const uint32_t e = ent[r];
            if (e != 0xffffffffu) {
                const uint32_t t = e >> kTileBits;
                const uint32_t pos = base[t] + rank[r];
                // the count pass saw the same contributions; the guard keeps a
                // record inside its tile's range whatever happens
                if (pos < end[t]) {
                    keys[pos] = e;
                    vals[pos] = make_float2(v0[r], v1[r]);
                }
            }
        }
        if (valid && dx_parts != nullptr) {
            if (PLANAR) {   // per-group partials, summed by the consumer
                float *o = dx_parts + ((size_t)g * cap + s) * 3;
                o[0] = d0;
                o[1] = d1;
                o[2] = d2;
            } else {        // accumulate into dx[n][3]
                unsafeAtomicAdd(dx_parts + 3 * s, d0);
                unsafeAtomicAdd(dx_parts + 3 * s + 1, d1);
                unsafeAtomicAdd(dx_parts + 3 * s + 2, d2);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- accumulate
__global__ void __launch_bounds__(kAccumBlock)
scatter_accum(int n_tiles, uint32_t n_entries, const uint32_t *__restrict__ start,
              const uint32_t *__restrict__ item_start, const uint32_t *__restrict__ n_items,
              const uint32_t *__restrict__ keys, const float2 *__restrict__ vals,
              float *__restrict__ dtable, float *__restrict__ partial) {
    extern __shared__ float acc[];    // [2 * kTileEntries]
    const uint32_t items = *n_items;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        // tile of this item: last t with item_start[t] <= it
        int lo = 0, hi = n_tiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_start[mid] <= it) lo = mid;
            else hi = mid - 1;
        }
        const int t = lo;
        const uint32_t first = it - item_start[t];
        const uint32_t r0 = start[t] + first * kItemRecords;
        const uint32_t r1e = r0 + kItemRecords;
        const uint32_t r1 = r1e < start[t + 1] ? r1e : start[t + 1];
        const bool owner = (item_start[t + 1] - item_start[t]) == 1u;
        for (int i = threadIdx.x; i < 2 * kTileEntries; i += blockDim.x) acc[i] = 0.f;
        __syncthreads();
        const uint32_t tbase = (uint32_t)t << kTileBits;
        // kUnroll records per thread are loaded before any is added, so that
        // each wave keeps several global loads in flight
        constexpr int kUnroll = 8;
        for (uint32_t r = r0 + threadIdx.x; r < r1; r += kUnroll * blockDim.x) {
            uint32_t loc[kUnroll];
            float2 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t ru = r + u * blockDim.x;
                loc[u] = 0xffffffffu;
                if (ru < r1) {
                    loc[u] = keys[ru] - tbase;
                    v[u] = vals[ru];
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (loc[u] < (uint32_t)kTileEntries) {   // every record of the range is in the tile
                    atomicAdd(&acc[2 * loc[u]], v[u].x);
                    atomicAdd(&acc[2 * loc[u] + 1], v[u].y);
                }
            }
        }
        __syncthreads();
        const uint32_t ne = (n_entries - tbase) < (uint32_t)kTileEntries ? (n_entries - tbase)
                                                                          : (uint32_t)kTileEntries;
        if (owner) {
            for (uint32_t i = threadIdx.x; i < 2 * ne; i += blockDim.x) {
                const float v = acc[i];
                if (v != 0.f) dtable[2 * (size_t)tbase + i] += v;
            }
        } else {
            float *slab = partial + (size_t)it * (2 * kTileEntries);
            for (uint32_t i = threadIdx.x; i < 2 * ne; i += blockDim.x) slab[i] = acc[i];
        }
        __syncthreads();
    }
}

// Adds the partial slabs of every split tile into the gradient table.
__global__ void __launch_bounds__(256)
scatter_reduce(int n_tiles, uint32_t n_entries, const uint32_t *__restrict__ item_start,
               const float *__restrict__ partial, float *__restrict__ dtable) {
    const int t = blockIdx.y;
    const uint32_t i0 = item_start[t], i1 = item_start[t + 1];
    if (i1 - i0 <= 1u) return;                 // single-item tiles are already added
    const uint32_t tbase = (uint32_t)t << kTileBits;
    const uint32_t ne2 = 2 * ((n_entries - tbase) < (uint32_t)kTileEntries ? (n_entries - tbase)
                                                                              : (uint32_t)kTileEntries);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne2; i += gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (uint32_t it = i0; it < i1; ++it) acc += partial[(size_t)it * (2 * kTileEntries) + i];
        if (acc != 0.f) dtable[2 * (size_t)tbase + i] += acc;
    }
}

nvr_status scatter_check(const GridParams &p) {
    const int nt = scatter_tiles(p);
    NVR_REQUIRE(nt >= 1 && nt <= 8192, NVR_EUNSUPPORTED, "binned scatter needs <= 8192 tiles");
    NVR_REQUIRE((p.L + kXcds - 1) / kXcds <= kMaxLpg, NVR_EUNSUPPORTED, "too many levels");
    return NVR_OK;
}

nvr_status launch_scatter(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                          const float *x, const void *table, const float *dfeat, float *dtable,
                          float *dx_parts, bool planar, void *ws, hipStream_t st) {
    if (cap <= 0) return NVR_OK;
    NVR_TRY(scatter_check(p));
    const int nt = scatter_tiles(p);
    ScatterWs w = carve_scatter(p, ws, cap);
    zero_u32<<<grid_for(nt + 1, 256, 64), 256, 0, st>>>(w.count, nt + 1);
    NVR_LAUNCHED();
    const unsigned chunks = grid_for(cap, kBinBlock, 512);
    const unsigned gr = chunks * kXcds;
    scatter_count<<<gr, kBinBlock, sizeof(uint32_t) * nt, st>>>(p, nt, n, n_dev, cap, x, w.count);
    NVR_LAUNCHED();
    scatter_scan<<<1, 1024, 0, st>>>(nt, w.count, w.start, w.cursor, w.item_start, w.n_items);
    NVR_LAUNCHED();
    const int lpg = (p.L + kXcds - 1) / kXcds;
    const size_t emit_lds = 3 * sizeof(uint32_t) * nt;
#define NVR_EMIT(PL, LP)                                                                       \
    scatter_emit<PL, LP><<<gr, kBinBlock, emit_lds, st>>>(p, nt, n, n_dev, cap, x,             \
                                                          (const uint32_t *)table, dfeat,       \
                                                          w.start, w.cursor, w.keys, w.vals,   \
                                                          dx_parts)
#define NVR_EMIT_L(PL)                                                                         \
    switch (lpg) {                                                                             \
    case 1: NVR_EMIT(PL, 1); break;                                                            \
    case 2: NVR_EMIT(PL, 2); break;                                                            \
    case 3: NVR_EMIT(PL, 3); break;                                                            \
    default: NVR_EMIT(PL, 4); break;                                                           \
    }
    if (planar) {
        NVR_EMIT_L(true)
    } else {
        NVR_EMIT_L(false)
    }
#undef NVR_EMIT_L
#undef NVR_EMIT
    NVR_LAUNCHED();
    const int64_t max_items = max_items_of(cap, p.L, nt);
    const unsigned ga = (unsigned)(max_items < 2048 ? max_items : 2048);
    static bool lds_ok = false;   // opt in to more than 64 KiB of dynamic LDS
    if (!lds_ok) {
        NVR_HIP(hipFuncSetAttribute((const void *)scatter_accum,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(float) * 2 * kTileEntries)));
        lds_ok = true;
    }
    scatter_accum<<<ga, kAccumBlock, sizeof(float) * 2 * kTileEntries, st>>>(
        nt, p.off[p.L], w.start, w.item_start, w.n_items, w.keys, w.vals, dtable, w.partial);
    NVR_LAUNCHED();
    scatter_reduce<<<dim3(2 * kTileEntries / 256, nt), 256, 0, st>>>(nt, p.off[p.L], w.item_start,
                                                                      w.partial, dtable);
    NVR_LAUNCHED();
    return NVR_OK;
}

}  // namespace nvr

using namespace nvr;

extern "C" size_t nvr_encode_bwd_workspace(const nvr_grid_desc *g, int64_t n) {
    if (check_grid(g) != NVR_OK || n < 0) return 0;
    return scatter_ws_bytes(make_grid_params(g), n);
}

extern "C" nvr_status nvr_encode_bwd_binned(const nvr_grid_desc *g, int64_t n, const float *x,
                                            const void *table, const float *dfeat, float *dtable,
                                            float *dx, void *workspace, nvr_stream stream) {
    clear_error();
    NVR_TRY(check_grid(g));
    NVR_REQUIRE(n >= 0 && n < (1ll << 31), NVR_EINVAL, "n out of range");
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(x && table && dfeat && dtable && workspace, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(aligned(x, 4) && aligned(table, 4) && aligned(dfeat, 4) && aligned(dtable, 8) &&
                    aligned(dx, 4) && aligned(workspace, 256),
                NVR_EINVAL, "misaligned array");
    const GridParams p = make_grid_params(g);
    NVR_TRY(scatter_check(p));
    NVR_REQUIRE((size_t)n * p.L * 8 < (1ull << 32), NVR_EINVAL, "too many contributions");
    return launch_scatter(p, n, nullptr, n, x, table, dfeat, dtable, dx, false, workspace,
                          hs(stream));
}
