// Binned backward of the hash encoding (table-gradient scatter without global
// float atomics per contribution).
//
// fp32 global atomics run at ~20 G/s on the whole device and serialise on the
// few entries of the coarse dense levels, which every sample hits; one step
// makes ~1.7 G of them.  Instead the scatter becomes a bucketed reduction:
//
//   count   every (sample, level, corner) contribution is assigned to the
//           table tile (2^tb entries, tb >= 10) holding its entry; per-workgroup
//           LDS histograms are added into per-tile counts;
//   scan    one workgroup turns the counts into tile ranges, resets the append
//           cursors and splits every tile into work items of <= 2^17 records
//           (fewer for small capacities; a hashed-level tile is one item, the
//           coarse dense tiles, which every sample hits, are split);
//   emit    the contributions (entry, w * dfeat_0, w * dfeat_1) are recomputed
//           and appended to their tile's range: ranks come from LDS counters,
//           one global atomic per (workgroup chunk, tile) reserves the space;
//           the position gradient (for the warp) is formed here as well.  A
//           record is 8 bytes: the two values rounded to nearest at
//           23 - kb mantissa bits, kb = ceil(tb / 2), whose low kb bits then
//           carry the entry's index inside the tile (high half in the first
//           value, low half in the second) -- the tile itself is implied by
//           the range the record sits in;
//   accum   one wavefront per work item sums its records into its own LDS
//           copy of the tile.  LDS float atomics cost about three cycles per
//           lane, so there are none: the lanes of one instruction that name the
//           same entry are serialised by a tag write and read-back (one winner
//           per entry and round does a plain read-add-write; a wave's LDS
//           operations complete in order).  A tile that is a single item is
//           added into the gradient table directly (it owns the tile), the
//           items of a split tile write their sums to partial slabs which a
//           last launch adds up per entry -- no global float atomics at all.
//
// Levels are split over the XCDs as in the forward (workgroup b serves level
// group b % 8) in count and emit.
#include "common.hpp"
#include "grid_dev.hpp"
#include "scatter_dev.hpp"

#include <atomic>

namespace nvr {

constexpr int kMinTileBits = 10;   // 8 KiB of float2 sums + 1 KiB of tags per wave
constexpr int kMaxTileBits = 14;
constexpr int kMaxTiles = 8192;
constexpr int kBinBlock = 256;     // count
constexpr int kEmitBlock = 1024;   // emit: samples per chunk (default; 512 and 256 also built)
constexpr int kMaxLpg = 4;   // levels per group (L <= 32)
constexpr int kMaxLevelTiles = 2048;   // tiles one level may span
// emit LDS: per-level tile counts / offsets and deltas (lt each), one partial
// per wave, and the staged records with their tiles (8 per sample)
static size_t emit_lds_bytes(int block, int lt) {
    return sizeof(uint32_t) * (2 * (size_t)lt + 16) + (sizeof(uint2) + sizeof(uint16_t)) * 8 * block;
}
constexpr size_t kRecPad = 512;   // records of padding after the record buffer (one accum window)

// Records per work item of a split tile: 2^17, or fewer (down to 2^13) when the
// capacity's records would make fewer than 2048 items, so that the coarse dense
// tiles of a small call (every sample hits them) are not summed by a few waves.
static uint32_t item_records(int64_t cap, int L) {
    const int64_t want = (int64_t)cap * L * 8 / 2048;
    uint32_t r = 1u << 13;
    while (r < (1u << 17) && (int64_t)(r << 1) <= want) r <<= 1;
    return r;
}

static int64_t max_items_of(int64_t cap, int L, int nt) {
    return (int64_t)cap * L * 8 / item_records(cap, L) + nt + 1;
}

// smallest tile size (>= 2^10 entries) that keeps the tile count <= 8192
static int tile_bits(const GridParams &p) {
    int tb = kMinTileBits;
    while (tb < kMaxTileBits && (((int64_t)p.off[p.L] + (1ll << tb) - 1) >> tb) > kMaxTiles) ++tb;
    return tb;
}

int scatter_tiles(const GridParams &p) {
    const int tb = tile_bits(p);
    return (int)(((int64_t)p.off[p.L] + (1ll << tb) - 1) >> tb);
}

static size_t accum_lds_bytes(int tb) { return (sizeof(float2) + 1) << tb; }

size_t scatter_ws_bytes(const GridParams &p, int64_t cap) {
    const int nt = scatter_tiles(p);
    const size_t max_rec = (size_t)cap * p.L * 8;
    size_t b = 0;
    b += sizeof(uint32_t) * (size_t)(4 * (nt + 1) + 4);  // counts, starts, cursors, items, n
    b = (b + 255) & ~size_t(255);
    b += sizeof(uint2) * (max_rec + kRecPad);            // packed records
    b = (b + 255) & ~size_t(255);
    b += (sizeof(float2) << tile_bits(p)) * (size_t)max_items_of(cap, p.L, nt);  // partial slabs
    return b;
}

struct ScatterWs {
    uint32_t *count, *start, *cursor, *item_start, *n_items;
    uint2 *rec;           // packed records
    float2 *partial;      // [max_items][tile entries]
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
    w.rec = (uint2 *)((char *)ws + b);
    b += sizeof(uint2) * (max_rec + kRecPad);
    b = (b + 255) & ~size_t(255);
    w.partial = (float2 *)((char *)ws + b);
    return w;
}

__global__ void zero_u32(uint32_t *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- count
__global__ void __launch_bounds__(kBinBlock)
scatter_count(GridParams p, int tb, int n_tiles, int64_t n, const int32_t *__restrict__ n_dev,
              int64_t cap, const float *__restrict__ x, uint32_t *__restrict__ tile_count) {
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
                for (int j = 0; j < 4; ++j) {   // an x edge's two corners: one tile but rarely
                    const uint32_t t0 = (p.off[l] + corner_index(p, l, lp, 2 * j)) >> tb;
                    const uint32_t t1 = (p.off[l] + corner_index(p, l, lp, 2 * j + 1)) >> tb;
                    atomicAdd(&hist[t0], t0 == t1 ? 2u : 1u);
                    if (t0 != t1) atomicAdd(&hist[t1], 1u);
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
             uint32_t *__restrict__ n_items, uint32_t item) {
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
        const uint32_t it = (c + item - 1) / item;
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
// Packed record: each value rounded to nearest (ties away from zero) at its
// low kb mantissa bits, which then hold half of the in-tile index.  A non-finite
// value stays non-finite.
__device__ inline uint32_t round_low_bits(float v, int kb) {
    const uint32_t b = __float_as_uint(v) + (1u << (kb - 1));
    return b & ~((1u << kb) - 1u);
}

__device__ inline uint2 pack_record(uint32_t loc, int kb, float v0, float v1) {
    const uint32_t m = (1u << kb) - 1u;
    return make_uint2(round_low_bits(v0, kb) | (loc >> kb), round_low_bits(v1, kb) | (loc & m));
}

// In-place exclusive prefix sum of a[0, n) by the whole workgroup (part holds
// one partial per wavefront).  Starts and ends with a barrier.
__device__ void block_exclusive_scan(uint32_t *a, int n, uint32_t *part) {
    __syncthreads();
    const int nt = blockDim.x;
    const int seg = (n + nt - 1) / nt;
    const int i0 = threadIdx.x * seg;
    const int i1 = i0 + seg < n ? i0 + seg : n;
    uint32_t s = 0;
    for (int i = i0; i < i1; ++i) s += a[i];
    // inclusive scan inside the wavefront
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(inc, d, 64);
        if (lane >= d) inc += v;
    }
    if (lane == 63) part[wave] = inc;
    __syncthreads();
    uint32_t run = inc - s;
    for (int w = 0; w < wave; ++w) run += part[w];
    for (int i = i0; i < i1; ++i) {
        const uint32_t c = a[i];
        a[i] = run;
        run += c;
    }
    __syncthreads();
}

// Position-gradient sum of one level: each corner's table pair (fp16)
// contracted with the feature gradient, weighted by the corner weight's
// derivative.  With a 16-byte aligned table (level slices start at multiples of
// 8 entries) the two corners of a cell edge along x come from one aligned
// 16-byte load, plus a 4-byte load in the cases where the edge straddles two
// groups of 4 entries, as in the forward gather.
__device__ __forceinline__ uint32_t word_of(const uint4 &q, uint32_t i) {
    const uint32_t lo = (i & 1u) ? q.y : q.x;
    const uint32_t hi = (i & 1u) ? q.w : q.z;
    return (i & 2u) ? hi : lo;
}

__device__ __forceinline__ float3 level_dx_sum(const uint32_t *__restrict__ table,
                                               const uint32_t (&ent)[8], bool quad,
                                               const LevelPos &lp, float g0, float g1) {
    uint32_t v[8];
    if (quad) {
        uint4 q[4];
        uint32_t far_v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = *reinterpret_cast<const uint4 *>(table + (ent[2 * j] & ~3u));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            far_v[j] = 0u;
            if ((ent[2 * j] ^ ent[2 * j + 1]) > 3u) far_v[j] = table[ent[2 * j + 1]];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[2 * j] = word_of(q[j], ent[2 * j] & 3u);
            v[2 * j + 1] = (ent[2 * j] ^ ent[2 * j + 1]) > 3u ? far_v[j]
                                                               : word_of(q[j], ent[2 * j + 1] & 3u);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = table[ent[k]];
    }
    float e0 = 0.f, e1 = 0.f, e2 = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float tg = f16_bits_to_f32((uint16_t)(v[k] & 0xffffu)) * g0 +
                         f16_bits_to_f32((uint16_t)(v[k] >> 16)) * g1;
        const float3 dw = corner_dweight(lp, k);
        e0 += dw.x * tg;
        e1 += dw.y * tg;
        e2 += dw.z * tg;
    }
    return make_float3(e0, e1, e2);
}

// The same sum from the derivatives the forward gather stored (three fp16
// pairs, one per axis: d feature 0 and d feature 1 in cell units).
__device__ __forceinline__ float3 stored_dx_sum(const uint32_t *__restrict__ j, float g0, float g1) {
    float e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t v = j[a];
        e[a] = f16_bits_to_f32((uint16_t)(v & 0xffffu)) * g0 + f16_bits_to_f32((uint16_t)(v >> 16)) * g1;
    }
    return make_float3(e[0], e[1], e[2]);
}

// One chunk of blockDim.x samples and one level at a time: the chunk's 8 records
// per sample are ranked within their tiles (LDS counters), space is reserved
// per tile with one global atomic, the records are staged in LDS in tile order
// and then written out by consecutive threads to consecutive positions, so
// that each tile's run is stored contiguously.  DX: the position gradient is
// formed as well (its own instantiation, so that the plain one keeps fewer
// registers).
template <int LPG, int BLOCK, bool DX>
__global__ void __launch_bounds__(BLOCK)
scatter_emit(GridParams p, int tb, int lt, int64_t n, const int32_t *__restrict__ n_dev,
             int64_t cap, const float *__restrict__ x, const uint32_t *__restrict__ table,
             const float *__restrict__ dfeat, uint32_t n_records, uint32_t *__restrict__ cursor,
             uint2 *__restrict__ recs, float *__restrict__ dx_parts,
             const uint32_t *__restrict__ jac) {
    extern __shared__ uint32_t lds[];
    uint32_t *hist = lds;                               // [lt] counts, then offsets
    uint32_t *delta = hist + lt;                        // [lt] global - local position
    uint32_t *part = delta + lt;                        // [16] one per wave
    uint2 *srec = reinterpret_cast<uint2 *>(part + 16);               // [8 * BLOCK] staged
    uint16_t *stile = reinterpret_cast<uint16_t *>(srec + 8 * BLOCK);  // their tiles - t_lo
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int lpg = LPG;
    const int kb = (tb + 1) >> 1;
    const bool quad = ((uintptr_t)table & 15u) == 0;   // level slices are 8-entry aligned
    for (int64_t c = blockIdx.x / kXcds; c * blockDim.x < count; c += chunks) {
        const int64_t s = c * blockDim.x + threadIdx.x;
        const bool valid = s < count;
        const int64_t left = count - c * blockDim.x;
        const uint32_t n_rec = 8u * (uint32_t)(left < (int64_t)blockDim.x ? left : blockDim.x);
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;
        float px = 0.f, py = 0.f, pz = 0.f;
        if (valid) {
            px = x[3 * s];
            py = x[3 * s + 1];
            pz = x[3 * s + 2];
        }
        for (int m = 0; m < LPG; ++m) {
            const int l = g + kXcds * m;
            if (l >= p.L) break;                       // the same for the whole workgroup
            const int t_lo = (int)((uint32_t)p.off[l] >> tb);
            const int n_lt = (int)((uint32_t)(p.off[l + 1] - 1) >> tb) - t_lo + 1;
            for (int t = threadIdx.x; t < n_lt; t += blockDim.x) hist[t] = 0u;
            __syncthreads();
            uint32_t ent[8], rank[8];
            float v0[8], v1[8];
            if (valid) {
                const LevelPos lp = level_pos(p, l, px, py, pz);
                const float *src = dfeat + ((size_t)g * cap + s) * (2 * lpg) + 2 * m;
                const float g0 = src[0], g1 = src[1];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float w = corner_weight(lp, k);
                    const uint32_t e = p.off[l] + corner_index(p, l, lp, k);
                    ent[k] = e;
                    v0[k] = w * g0;
                    v1[k] = w * g1;
                }
                float3 ed = make_float3(0.f, 0.f, 0.f);
                if (DX)
                    ed = jac != nullptr ? stored_dx_sum(jac + ((size_t)g * cap + s) * (3 * LPG) + 3 * m, g0, g1)
                                        : level_dx_sum(table, ent, quad, lp, g0, g1);
                // ranks inside the tiles; the two corners of an x edge (2j, 2j + 1)
                // fall into one tile but rarely, and then take one counter update
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t0 = (int)(ent[2 * j] >> tb) - t_lo;
                    const int t1 = (int)(ent[2 * j + 1] >> tb) - t_lo;
                    const uint32_t r = atomicAdd(&hist[t0], t0 == t1 ? 2u : 1u);
                    rank[2 * j] = r;
                    rank[2 * j + 1] = t0 == t1 ? r + 1u : atomicAdd(&hist[t1], 1u);
                }
                if (DX) {
                    if (lp.inside[0]) d0 += ed.x * p.s_hi[l][0];
                    if (lp.inside[1]) d1 += ed.y * p.s_hi[l][1];
                    if (lp.inside[2]) d2 += ed.z * p.s_hi[l][2];
                }
            }
            __syncthreads();
            for (int t = threadIdx.x; t < n_lt; t += blockDim.x) {
                const uint32_t h = hist[t];
                delta[t] = h ? atomicAdd(&cursor[t_lo + t], h) : 0u;
            }
            block_exclusive_scan(hist, n_lt, part);
            for (int t = threadIdx.x; t < n_lt; t += blockDim.x) delta[t] -= hist[t];
            if (valid) {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t slot = hist[(int)(ent[k] >> tb) - t_lo] + rank[k];
                    srec[slot] = pack_record(ent[k] & ((1u << tb) - 1u), kb, v0[k], v1[k]);
                    stile[slot] = (uint16_t)((int)(ent[k] >> tb) - t_lo);
                }
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < n_rec; i += blockDim.x) {
                // the count pass saw the same contributions, so pos stays inside
                // the tile's range; the bound keeps every store inside the buffer
                const uint32_t pos = delta[stile[i]] + i;
                if (pos < n_records) recs[pos] = srec[i];
            }
            __syncthreads();
        }
        if (valid && DX) {   // per-group partials, summed by the consumer
            float *o = dx_parts + ((size_t)g * cap + s) * 3;
            o[0] = d0;
            o[1] = d1;
            o[2] = d2;
        }
    }
}

// ---------------------------------------------------------------- accumulate
// One wavefront (the whole workgroup) per work item.
__global__ void __launch_bounds__(64)
scatter_accum(int tb, int n_tiles, uint32_t n_entries, const uint32_t *__restrict__ start,
              const uint32_t *__restrict__ item_start, const uint32_t *__restrict__ n_items,
              const uint2 *__restrict__ recs, float2 *__restrict__ dtable,
              float2 *__restrict__ partial, uint32_t item, int dense_tiles) {
    extern __shared__ float2 acc[];                                   // [te] sums
    const uint32_t te = 1u << tb;
    uint8_t *tag = reinterpret_cast<uint8_t *>(acc + te);            // [te]
    const uint32_t lane = threadIdx.x;
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
        const uint32_t r0 = start[t] + first * item;
        const uint32_t r1e = r0 + item;
        const uint32_t r1 = r1e < start[t + 1] ? r1e : start[t + 1];
        const bool owner = (item_start[t + 1] - item_start[t]) == 1u;
        for (uint32_t i = lane; i < te; i += 64) acc[i] = make_float2(0.f, 0.f);
        const uint32_t tbase = (uint32_t)t << tb;
        // Each lane takes kPer consecutive records of a 64 * kPer window (four
        // 16-byte loads), so a run of equal entries -- consecutive samples in
        // one coarse cell -- spreads over the rounds of one lane instead of the
        // lanes of one instruction.  Windows start 8-aligned at or below r0;
        // records outside [r0, r1) are masked off and the buffer carries one
        // window of padding.  The next window is loaded while the current one
        // is added.
        constexpr uint32_t kPer = 8;
        constexpr uint32_t kWin = 64u * kPer;
        const int kb = (tb + 1) >> 1;
        const uint32_t kmask = (1u << kb) - 1u;
        const uint32_t b0 = r0 & ~(kPer - 1u);
        uint4 qa, qb, qc, qd;
        {
            const uint4 *q = reinterpret_cast<const uint4 *>(recs + b0 + lane * kPer);
            qa = q[0];
            qb = q[1];
            qc = q[2];
            qd = q[3];
        }
        for (uint32_t base = b0; base < r1; base += kWin) {
            const uint32_t hw[kPer] = {qa.x, qa.z, qb.x, qb.z, qc.x, qc.z, qd.x, qd.z};
            const uint32_t lw[kPer] = {qa.y, qa.w, qb.y, qb.w, qc.y, qc.w, qd.y, qd.w};
            const uint32_t nb = base + kWin;
            if (nb < r1) {
                const uint4 *q = reinterpret_cast<const uint4 *>(recs + nb + lane * kPer);
                qa = q[0];
                qb = q[1];
                qc = q[2];
                qd = q[3];
            }
            uint32_t key[kPer];
            float v0[kPer], v1[kPer];
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                key[u] = tbase + (((hw[u] & kmask) << kb) | (lw[u] & kmask));
                v0[u] = __uint_as_float(hw[u] & ~kmask);
                v1[u] = __uint_as_float(lw[u] & ~kmask);
            }
            // one round per record slot u: every pending lane writes its lane id
            // to the tag of its entry and reads it back; exactly one lane per
            // entry sees its own id and adds.  The few losers (two lanes naming
            // one entry) are retried after all slots had their first round,
            // and only in slots that still have pending lanes.
            uint32_t loc[kPer];
            bool pend[kPer];
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                const uint32_t rec = base + lane * kPer + u;
                loc[u] = key[u] - tbase;
                // every record of the range is in the tile; the bound is a guard
                pend[u] = rec >= r0 && rec < r1 && loc[u] < te;
            }
            // in the dense levels (tiles below dense_tiles) consecutive samples in
            // one coarse cell leave a lane's window with the records of an x edge
            // alternating (A B A B ...): the lane first sums the records of one
            // entry that are one or two slots apart, so that the entry takes one
            // round in this lane instead of several
            if (t < dense_tiles)
#pragma unroll
            for (uint32_t u = 1; u < kPer; ++u) {
#pragma unroll
                for (uint32_t d = 1; d <= 2; ++d) {
                    if (d > u) continue;
                    const uint32_t w = u - d;
                    if (pend[w] && pend[u] && loc[w] == loc[u]) {
                        v0[u] += v0[w];
                        v1[u] += v1[w];
                        pend[w] = false;
                    }
                }
            }
            auto round = [&](uint32_t u) {
                // wavefront-scope relaxed atomics: plain LDS byte accesses that
                // the compiler may neither drop nor merge
                if (pend[u])
                    __hip_atomic_store(tag + loc[u], (uint8_t)lane, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
                if (pend[u] && __hip_atomic_load(tag + loc[u], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WAVEFRONT) == (uint8_t)lane) {
                    float2 a = acc[loc[u]];
                    a.x += v0[u];
                    a.y += v1[u];
                    acc[loc[u]] = a;
                    pend[u] = false;
                }
            };
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) round(u);
            bool left = false;
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) left |= pend[u];
            while (__ballot(left)) {
#pragma unroll
                for (uint32_t u = 0; u < kPer; ++u)
                    if (__ballot(pend[u])) round(u);
                left = false;
#pragma unroll
                for (uint32_t u = 0; u < kPer; ++u) left |= pend[u];
            }
        }
        const uint32_t ne = (n_entries - tbase) < te ? (n_entries - tbase) : te;
        if (owner) {
            // 16 entries per lane at a time: all table loads are issued before
            // the first add (indices past the tile end are clamped, not stored)
            for (uint32_t i0 = 0; i0 < ne; i0 += 64u * 16u) {
                float2 a[16], d[16];
#pragma unroll
                for (uint32_t j = 0; j < 16; ++j) {
                    const uint32_t i = i0 + 64u * j + lane;
                    const uint32_t ic = i < ne ? i : ne - 1u;
                    a[j] = acc[ic];
                    d[j] = dtable[tbase + ic];
                }
#pragma unroll
                for (uint32_t j = 0; j < 16; ++j) {
                    const uint32_t i = i0 + 64u * j + lane;
                    if (i < ne && (a[j].x != 0.f || a[j].y != 0.f))
                        dtable[tbase + i] = make_float2(d[j].x + a[j].x, d[j].y + a[j].y);
                }
            }
        } else {
            float2 *slab = partial + (size_t)it * te;
            for (uint32_t i = lane; i < ne; i += 64) slab[i] = acc[i];
        }
    }
}

// Adds the partial slabs of every split tile into the gradient table.
__global__ void __launch_bounds__(256)
scatter_reduce(int tb, uint32_t n_entries, const uint32_t *__restrict__ item_start,
               const float2 *__restrict__ partial, float2 *__restrict__ dtable) {
    const int t = blockIdx.y;
    const uint32_t i0 = item_start[t], i1 = item_start[t + 1];
    if (i1 - i0 <= 1u) return;                 // single-item tiles are already added
    const uint32_t te = 1u << tb;
    const uint32_t tbase = (uint32_t)t << tb;
    const uint32_t ne = (n_entries - tbase) < te ? (n_entries - tbase) : te;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += gridDim.x * blockDim.x) {
        float a0 = 0.f, a1 = 0.f;
        for (uint32_t it = i0; it < i1; ++it) {
            const float2 v = partial[(size_t)it * te + i];
            a0 += v.x;
            a1 += v.y;
        }
        if (a0 != 0.f || a1 != 0.f) {
            float2 d = dtable[tbase + i];
            d.x += a0;
            d.y += a1;
            dtable[tbase + i] = d;
        }
    }
}

nvr_status scatter_check(const GridParams &p) {
    const int nt = scatter_tiles(p);
    NVR_REQUIRE(nt >= 1 && nt <= kMaxTiles, NVR_EUNSUPPORTED,
                "binned scatter needs <= 8192 tiles of <= 2^14 entries");
    NVR_REQUIRE((p.L + kXcds - 1) / kXcds <= kMaxLpg, NVR_EUNSUPPORTED, "too many levels");
    const int tb = tile_bits(p);
    for (int l = 0; l < p.L; ++l)
        NVR_REQUIRE(((p.off[l + 1] - 1) >> tb) - (p.off[l] >> tb) + 1 <= kMaxLevelTiles,
                    NVR_EUNSUPPORTED, "a level spans too many scatter tiles");
    return NVR_OK;
}

static int level_tiles(const GridParams &p, int tb) {
    int most = 1;
    for (int l = 0; l < p.L; ++l) {
        const int n = (int)(((p.off[l + 1] - 1) >> tb) - (p.off[l] >> tb) + 1);
        most = n > most ? n : most;
    }
    return most;
}

TileCounter scatter_counter(const GridParams &p, void *ws) {
    const int tb = tile_bits(p);
    return TileCounter{(uint32_t *)ws, tb, level_tiles(p, tb)};
}

nvr_status launch_counter_reset(const GridParams &p, void *ws, hipStream_t st) {
    const int nt = scatter_tiles(p);
    zero_u32<<<grid_for(nt + 1, 256, 64), 256, 0, st>>>((uint32_t *)ws, nt + 1);
    NVR_LAUNCHED();
    return NVR_OK;
}

nvr_status launch_scatter(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                          const float *x, const void *table, const float *dfeat, float *dtable,
                          float *dx_parts, void *ws, hipStream_t st, bool counted,
                          int emit_chunks, int emit_block, const uint32_t *jac,
                          const ScatterTail *tail) {
    if (cap <= 0) return NVR_OK;
    NVR_TRY(scatter_check(p));
    const int tb = tile_bits(p);
    const int nt = scatter_tiles(p);
    ScatterWs w = carve_scatter(p, ws, cap);
    const uint32_t n_records = (uint32_t)((uint64_t)cap * p.L * 8 < 0xffffffffull
                                              ? (uint64_t)cap * p.L * 8 : 0xffffffffull);
    const int eb = emit_block == 512 || emit_block == 256 ? emit_block : kEmitBlock;
    const unsigned gre = grid_for(cap, eb, emit_chunks > 0 ? emit_chunks : 64) * kXcds;
    const int lt = level_tiles(p, tb);
    const size_t elds = emit_lds_bytes(eb, lt);
    if (!counted) {
        zero_u32<<<grid_for(nt + 1, 256, 64), 256, 0, st>>>(w.count, nt + 1);
        NVR_LAUNCHED();
        const unsigned gr = grid_for(cap, kBinBlock, 512) * kXcds;
        scatter_count<<<gr, kBinBlock, sizeof(uint32_t) * nt, st>>>(p, tb, nt, n, n_dev, cap, x,
                                                                      w.count);
        NVR_LAUNCHED();
    }
    scatter_scan<<<1, 1024, 0, st>>>(nt, w.count, w.start, w.cursor, w.item_start, w.n_items,
                                     item_records(cap, p.L));
    NVR_LAUNCHED();
    const int lpg = (p.L + kXcds - 1) / kXcds;
#define NVR_EMIT_DX(LP, DXV)                                                                   \
    do {                                                                                       \
        if (eb == 512)                                                                         \
            scatter_emit<LP, 512, DXV><<<gre, 512, elds, st>>>(p, tb, lt, n, n_dev, cap, x,    \
                (const uint32_t *)table, dfeat, n_records, w.cursor, w.rec, dx_parts, jac);    \
        else if (eb == 256)                                                                    \
            scatter_emit<LP, 256, DXV><<<gre, 256, elds, st>>>(p, tb, lt, n, n_dev, cap, x,    \
                (const uint32_t *)table, dfeat, n_records, w.cursor, w.rec, dx_parts, jac);    \
        else                                                                                   \
            scatter_emit<LP, kEmitBlock, DXV><<<gre, kEmitBlock, elds, st>>>(p, tb, lt, n,     \
                n_dev, cap, x, (const uint32_t *)table, dfeat, n_records, w.cursor, w.rec,     \
                dx_parts, jac);                                                                \
    } while (0)
#define NVR_EMIT(LP)                                                                           \
    do {                                                                                       \
        if (dx_parts != nullptr) NVR_EMIT_DX(LP, true);                                        \
        else NVR_EMIT_DX(LP, false);                                                           \
    } while (0)
    // opt in to more than 64 KiB of dynamic LDS, once per device
    int dev = 0;
    NVR_HIP(hipGetDevice(&dev));
    static std::atomic<uint64_t> emit_lds_ok{0}, accum_lds_ok{0};
    const uint64_t dev_bit = 1ull << (dev & 63);
    if (!(emit_lds_ok.load() & dev_bit)) {
        const int most = (int)emit_lds_bytes(kEmitBlock, kMaxLevelTiles);
#define NVR_EMIT_FNS(DXV)                                                                      \
    (const void *)scatter_emit<1, kEmitBlock, DXV>, (const void *)scatter_emit<2, kEmitBlock, DXV>, \
        (const void *)scatter_emit<3, kEmitBlock, DXV>,                                        \
        (const void *)scatter_emit<4, kEmitBlock, DXV>, (const void *)scatter_emit<1, 512, DXV>, \
        (const void *)scatter_emit<2, 512, DXV>, (const void *)scatter_emit<3, 512, DXV>,      \
        (const void *)scatter_emit<4, 512, DXV>, (const void *)scatter_emit<1, 256, DXV>,      \
        (const void *)scatter_emit<2, 256, DXV>, (const void *)scatter_emit<3, 256, DXV>,      \
        (const void *)scatter_emit<4, 256, DXV>
        const void *fns[] = {NVR_EMIT_FNS(false), NVR_EMIT_FNS(true)};
#undef NVR_EMIT_FNS
        for (const void *f : fns)
            NVR_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, most));
        emit_lds_ok.fetch_or(dev_bit);
    }
    switch (lpg) {
    case 1: NVR_EMIT(1); break;
    case 2: NVR_EMIT(2); break;
    case 3: NVR_EMIT(3); break;
    default: NVR_EMIT(4); break;
    }
#undef NVR_EMIT
#undef NVR_EMIT_DX
    NVR_LAUNCHED();
    if (dtable == nullptr) return NVR_OK;   // scan + emit only
    const int64_t max_items = max_items_of(cap, p.L, nt);
    const unsigned ga = (unsigned)(max_items < 65535 ? max_items : 65535);
    const size_t acc_lds = accum_lds_bytes(tb);
    if (acc_lds > 65536 && !(accum_lds_ok.load() & dev_bit)) {
        NVR_HIP(hipFuncSetAttribute((const void *)scatter_accum,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)accum_lds_bytes(kMaxTileBits)));
        accum_lds_ok.fetch_or(dev_bit);
    }
    int dense_end = 0;   // levels are stored coarse to fine, the dense ones first
    while (dense_end < p.L && p.dense[dense_end]) ++dense_end;
    const int dense_tiles = (int)(((int64_t)p.off[dense_end] + (1 << tb) - 1) >> tb);
    hipStream_t sa = st;
    if (tail != nullptr) {
        NVR_HIP(hipEventRecord(tail->fork, st));
        NVR_HIP(hipStreamWaitEvent(tail->stream, tail->fork, 0));
        sa = tail->stream;
    }
    scatter_accum<<<ga, 64, acc_lds, sa>>>(tb, nt, p.off[p.L], w.start, w.item_start, w.n_items,
                                           w.rec, (float2 *)dtable, w.partial,
                                           item_records(cap, p.L), dense_tiles);
    NVR_LAUNCHED();
    scatter_reduce<<<dim3(((1u << tb) + 255) / 256, nt), 256, 0, sa>>>(
        tb, p.off[p.L], w.item_start, w.partial, (float2 *)dtable);
    NVR_LAUNCHED();
    return NVR_OK;
}

// ---------------------------------------------------------------- deterministic variant
// The same records and sums in an order fixed by the inputs alone.  A tile's
// range holds its levels in increasing order; a level's records are ordered by
// chunk (kDetBlock consecutive samples), inside a chunk by wavefront, then by
// corner, then by lane.  Counts per (chunk, level, tile) are formed first and
// scanned over the chunks, so no range is reserved in a race; ranks inside a
// wavefront come from ballots; the accumulation gives every entry of a tile
// to one lane, which adds that entry's records in range order.  Split tiles
// are added up slab by slab in item order as before.
constexpr int kDetBlock = 512;
constexpr int kDetWaves = kDetBlock / 64;

struct DetSeg {
    int at[NVR_MAX_LEVELS + 1];   // first column of level l's tiles in a count row
};

static DetSeg det_segments(const GridParams &p, int tb) {
    DetSeg sg;
    int s = 0;
    for (int l = 0; l < p.L; ++l) {
        sg.at[l] = s;
        s += (int)(((p.off[l + 1] - 1) >> tb) - (p.off[l] >> tb) + 1);
    }
    for (int l = p.L; l <= NVR_MAX_LEVELS; ++l) sg.at[l] = s;
    return sg;
}

static size_t det_lds_bytes(int lt) {
    return sizeof(uint32_t) * ((size_t)(2 + kDetWaves) * lt + 16) +
           (sizeof(uint2) + sizeof(uint16_t)) * 8 * kDetBlock;
}

// The chunk columns of the count rows are scanned in kSegParts slices of
// consecutive chunks (slice sums, then per-slice bases, then the slices).
constexpr int kSegParts = 64;

size_t scatter_det_ws_bytes(const GridParams &p, int64_t cap) {
    const int tb = tile_bits(p);
    const DetSeg sg = det_segments(p, tb);
    const int64_t nc = (cap + kDetBlock - 1) / kDetBlock;
    return ((scatter_ws_bytes(p, cap) + 255) & ~size_t(255)) +
           sizeof(uint32_t) * ((size_t)nc * sg.at[p.L] + 2 * (size_t)kSegParts * sg.at[p.L]);
}

// seg[c][sg.at[l] + j] = records of chunk c that level l puts into its j-th
// tile; tile_count[t] += the same (integer sums: order-free).
template <int LPG>
__global__ void __launch_bounds__(kDetBlock)
det_count(GridParams p, int tb, DetSeg sg, int64_t n, const int32_t *__restrict__ n_dev,
          int64_t cap, const float *__restrict__ x, uint32_t *__restrict__ seg,
          uint32_t *__restrict__ tile_count) {
    extern __shared__ uint32_t hist[];
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int S = sg.at[p.L];
    for (int64_t c = blockIdx.x / kXcds; c * kDetBlock < count; c += chunks) {
        const int64_t s = c * kDetBlock + threadIdx.x;
        const bool valid = s < count;
        float px = 0.f, py = 0.f, pz = 0.f;
        if (valid) {
            px = x[3 * s];
            py = x[3 * s + 1];
            pz = x[3 * s + 2];
        }
        for (int m = 0; m < LPG; ++m) {
            const int l = g + kXcds * m;
            if (l >= p.L) break;
            const int t_lo = (int)(p.off[l] >> tb);
            const int n_lt = (int)((p.off[l + 1] - 1) >> tb) - t_lo + 1;
            for (int t = threadIdx.x; t < n_lt; t += kDetBlock) hist[t] = 0u;
            __syncthreads();
            if (valid) {
                const LevelPos lp = level_pos(p, l, px, py, pz);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    atomicAdd(&hist[(int)((p.off[l] + corner_index(p, l, lp, k)) >> tb) - t_lo], 1u);
            }
            __syncthreads();
            uint32_t *row = seg + (size_t)c * S + sg.at[l];
            for (int t = threadIdx.x; t < n_lt; t += kDetBlock) {
                const uint32_t h = hist[t];
                row[t] = h;
                if (h) atomicAdd(&tile_count[t_lo + t], h);
            }
            __syncthreads();
        }
    }
}

// The position of every (chunk, level, tile) run: a tile's range holds its
// levels in increasing order and, inside each, its chunks in order, so seg
// becomes the exclusive prefix of its column plus the tile's start.  Three
// passes over kSegParts slices of consecutive chunks: the slice sums of every
// column, the slices' bases (one thread per tile, through its levels), and the
// prefixes inside the slices.  Integer sums: the result is the one serial
// walk over the chunks would give.
__device__ __forceinline__ void seg_slice(int64_t nc, int part, int64_t *c0, int64_t *c1) {
    const int64_t per = (nc + kSegParts - 1) / kSegParts;
    *c0 = per * part < nc ? per * part : nc;
    *c1 = per * (part + 1) < nc ? per * (part + 1) : nc;
}

__global__ void __launch_bounds__(256)
det_seg_sums(DetSeg sg, int L, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
             const uint32_t *__restrict__ seg, uint32_t *__restrict__ psum) {
    const int S = sg.at[L];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * kSegParts) return;
    const int j = (int)(i % S), part = (int)(i / S);
    const int64_t nc = (count_of(n, n_dev, cap) + kDetBlock - 1) / kDetBlock;
    int64_t c0, c1;
    seg_slice(nc, part, &c0, &c1);
    uint32_t a = 0u;
    for (int64_t c = c0; c < c1; ++c) a += seg[c * S + j];
    psum[(size_t)part * S + j] = a;
}

__global__ void __launch_bounds__(256)
det_seg_bases(GridParams p, int tb, DetSeg sg, int n_tiles, const uint32_t *__restrict__ start,
              const uint32_t *__restrict__ psum, uint32_t *__restrict__ pbase) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const size_t S = (size_t)sg.at[p.L];
    uint32_t run = start[t];
    for (int l = 0; l < p.L; ++l) {
        const int t_lo = (int)(p.off[l] >> tb), t_hi = (int)((p.off[l + 1] - 1) >> tb);
        if (t < t_lo || t > t_hi) continue;
        const size_t j = (size_t)sg.at[l] + (t - t_lo);
        for (int part = 0; part < kSegParts; ++part) {
            pbase[part * S + j] = run;
            run += psum[part * S + j];
        }
    }
}

__global__ void __launch_bounds__(256)
det_seg_apply(DetSeg sg, int L, int64_t n, const int32_t *__restrict__ n_dev, int64_t cap,
              const uint32_t *__restrict__ pbase, uint32_t *__restrict__ seg) {
    const int S = sg.at[L];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * kSegParts) return;
    const int j = (int)(i % S), part = (int)(i / S);
    const int64_t nc = (count_of(n, n_dev, cap) + kDetBlock - 1) / kDetBlock;
    int64_t c0, c1;
    seg_slice(nc, part, &c0, &c1);
    uint32_t run = pbase[(size_t)part * S + j];
    for (int64_t c = c0; c < c1; ++c) {
        const uint32_t v = seg[c * S + j];
        seg[c * S + j] = run;
        run += v;
    }
}

template <int LPG>
__global__ void __launch_bounds__(kDetBlock)
det_emit(GridParams p, int tb, int lt, DetSeg sg, int64_t n, const int32_t *__restrict__ n_dev,
         int64_t cap, const float *__restrict__ x, const uint32_t *__restrict__ table,
         const float *__restrict__ dfeat, uint32_t n_records, const uint32_t *__restrict__ seg,
         uint2 *__restrict__ recs, float *__restrict__ dx_parts, const uint32_t *__restrict__ jac) {
    extern __shared__ uint32_t lds[];
    uint32_t *hist = lds;                               // [lt] chunk totals, then bases
    uint32_t *delta = hist + lt;                        // [lt] global - local position
    uint32_t *wc = delta + lt;                          // [waves][lt] counts, then prefixes
    uint32_t *part = wc + kDetWaves * lt;               // [16]
    uint2 *srec = reinterpret_cast<uint2 *>(part + 16);                   // [8 * block]
    uint16_t *stile = reinterpret_cast<uint16_t *>(srec + 8 * kDetBlock);  // their tiles - t_lo
    const int64_t count = count_of(n, n_dev, cap);
    const int g = blockIdx.x % kXcds;
    const int64_t chunks = gridDim.x / kXcds;
    const int kb = (tb + 1) >> 1;
    const bool quad = ((uintptr_t)table & 15u) == 0;   // level slices are 8-entry aligned
    const int S = sg.at[p.L];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t c = blockIdx.x / kXcds; c * kDetBlock < count; c += chunks) {
        const int64_t s = c * kDetBlock + threadIdx.x;
        const bool valid = s < count;
        const int64_t left = count - c * kDetBlock;
        const uint32_t n_rec = 8u * (uint32_t)(left < (int64_t)kDetBlock ? left : kDetBlock);
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;
        float px = 0.f, py = 0.f, pz = 0.f;
        if (valid) {
            px = x[3 * s];
            py = x[3 * s + 1];
            pz = x[3 * s + 2];
        }
        for (int m = 0; m < LPG; ++m) {
            const int l = g + kXcds * m;
            if (l >= p.L) break;
            const int t_lo = (int)(p.off[l] >> tb);
            const int n_lt = (int)((p.off[l + 1] - 1) >> tb) - t_lo + 1;
            for (int t = threadIdx.x; t < kDetWaves * n_lt; t += kDetBlock) wc[t] = 0u;
            __syncthreads();
            uint32_t ent[8], rank[8];
            int key[8];
            float v0[8], v1[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                key[k] = -1;
                rank[k] = 0u;
            }
            if (valid) {
                const LevelPos lp = level_pos(p, l, px, py, pz);
                const float *src = dfeat + ((size_t)g * cap + s) * (2 * LPG) + 2 * m;
                const float g0 = src[0], g1 = src[1];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float w = corner_weight(lp, k);
                    const uint32_t e = p.off[l] + corner_index(p, l, lp, k);
                    ent[k] = e;
                    key[k] = (int)(e >> tb) - t_lo;
                    v0[k] = w * g0;
                    v1[k] = w * g1;
                }
                float3 ed = make_float3(0.f, 0.f, 0.f);
                if (dx_parts != nullptr)
                    ed = jac != nullptr ? stored_dx_sum(jac + ((size_t)g * cap + s) * (3 * LPG) + 3 * m, g0, g1)
                                        : level_dx_sum(table, ent, quad, lp, g0, g1);
                if (dx_parts != nullptr) {
                    if (lp.inside[0]) d0 += ed.x * p.s_hi[l][0];
                    if (lp.inside[1]) d1 += ed.y * p.s_hi[l][1];
                    if (lp.inside[2]) d2 += ed.z * p.s_hi[l][2];
                }
            }
            // stable ranks inside the wavefront, corner-major then lane order;
            // the wavefront's running count per tile lives in its own LDS row.
            // Dense levels name few tiles per instruction: one round per tile
            // present.  Hashed levels name up to 64: each lane counts the lanes
            // below it with its tile (and all lanes with it) by reading every
            // lane's tile through the scalar unit, and the first lane of each
            // tile advances the row.  Both give the same ranks.
            uint32_t *mine = wc + wave * n_lt;
            if (p.dense[l]) {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    uint64_t todo = __ballot(key[k] >= 0);
                    while (todo) {
                        const int leader = __ffsll((unsigned long long)todo) - 1;
                        const int K = __shfl(key[k], leader, 64);
                        const uint64_t same = __ballot(key[k] == K);
                        const uint32_t base = __hip_atomic_load(mine + K, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_WAVEFRONT);
                        if (key[k] == K) rank[k] = base + (uint32_t)__popcll(same & below);
                        if (lane == leader)
                            __hip_atomic_store(mine + K, base + (uint32_t)__popcll(same),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                        todo &= ~same;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    uint32_t lower = 0u, total = 0u;
                    for (int j = 0; j < 64; ++j) {
                        const int kj = __builtin_amdgcn_readlane(key[k], j);
                        const bool eq = kj == key[k];
                        total += eq ? 1u : 0u;
                        lower += (eq && j < lane) ? 1u : 0u;
                    }
                    const bool has = key[k] >= 0;
                    uint32_t base = 0u;
                    if (has)
                        base = __hip_atomic_load(mine + key[k], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
                    if (has) rank[k] = base + lower;
                    if (has && lower == 0u)
                        __hip_atomic_store(mine + key[k], base + total, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            }
            __syncthreads();
            // per tile: exclusive prefix over the wavefronts (in place) and chunk total
            for (int t = threadIdx.x; t < n_lt; t += kDetBlock) {
                uint32_t run = 0u;
                for (int w = 0; w < kDetWaves; ++w) {
                    const uint32_t v = wc[w * n_lt + t];
                    wc[w * n_lt + t] = run;
                    run += v;
                }
                hist[t] = run;
                delta[t] = seg[(size_t)c * S + sg.at[l] + t];
            }
            block_exclusive_scan(hist, n_lt, part);
            for (int t = threadIdx.x; t < n_lt; t += kDetBlock) delta[t] -= hist[t];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (key[k] >= 0) {
                    const uint32_t slot = hist[key[k]] + mine[key[k]] + rank[k];
                    srec[slot] = pack_record(ent[k] & ((1u << tb) - 1u), kb, v0[k], v1[k]);
                    stile[slot] = (uint16_t)key[k];
                }
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < n_rec; i += kDetBlock) {
                const uint32_t pos = delta[stile[i]] + i;
                if (pos < n_records) recs[pos] = srec[i];
            }
            __syncthreads();
        }
        if (valid && dx_parts != nullptr) {
            float *o = dx_parts + ((size_t)g * cap + s) * 3;
            o[0] = d0;
            o[1] = d1;
            o[2] = d2;
        }
    }
}

// One wavefront per work item; lane j owns the tile entries with index j mod
// 64 and adds their records in range order (LDS adds of one lane issue in
// program order).  A window of 512 records is staged in LDS and read by every
// lane.
// The deterministic accumulate for tiles of at most kDetFastEntries entries:
// the same windows and rounds as scatter_accum, but the lane that adds an
// entry's record in a round is chosen by an integer minimum over the lanes
// naming it (tags reset, then ds_min of the lane id, then read back), so the
// order in which an entry's records are added depends only on their order in
// the record buffer, which the deterministic emit fixes.
constexpr uint32_t kDetFastEntries = 8192;
__global__ void __launch_bounds__(64)
det_accum_min(int tb, int n_tiles, uint32_t n_entries, const uint32_t *__restrict__ start,
              const uint32_t *__restrict__ item_start, const uint32_t *__restrict__ n_items,
              const uint2 *__restrict__ recs, float2 *__restrict__ dtable,
              float2 *__restrict__ partial, uint32_t item) {
    extern __shared__ float2 acc[];                                   // [te] sums
    const uint32_t te = 1u << tb;
    uint32_t *tag = reinterpret_cast<uint32_t *>(acc + te);          // [te]
    const uint32_t lane = threadIdx.x;
    const uint32_t items = *n_items;
    const int kb = (tb + 1) >> 1;
    const uint32_t kmask = (1u << kb) - 1u;
    constexpr uint32_t kPer = 8;
    constexpr uint32_t kWin = 64u * kPer;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        int lo = 0, hi = n_tiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_start[mid] <= it) lo = mid;
            else hi = mid - 1;
        }
        const int t = lo;
        const uint32_t first = it - item_start[t];
        const uint32_t r0 = start[t] + first * item;
        const uint32_t r1e = r0 + item;
        const uint32_t r1 = r1e < start[t + 1] ? r1e : start[t + 1];
        const bool owner = (item_start[t + 1] - item_start[t]) == 1u;
        for (uint32_t i = lane; i < te; i += 64) acc[i] = make_float2(0.f, 0.f);
        const uint32_t tbase = (uint32_t)t << tb;
        const uint32_t b0 = r0 & ~(kPer - 1u);
        for (uint32_t base = b0; base < r1; base += kWin) {
            const uint4 *q = reinterpret_cast<const uint4 *>(recs + base + lane * kPer);
            const uint4 qv[4] = {q[0], q[1], q[2], q[3]};
            const uint32_t hw[kPer] = {qv[0].x, qv[0].z, qv[1].x, qv[1].z,
                                       qv[2].x, qv[2].z, qv[3].x, qv[3].z};
            const uint32_t lw[kPer] = {qv[0].y, qv[0].w, qv[1].y, qv[1].w,
                                       qv[2].y, qv[2].w, qv[3].y, qv[3].w};
            uint32_t loc[kPer];
            float v0[kPer], v1[kPer];
            bool pend[kPer];
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                const uint32_t rec = base + lane * kPer + u;
                loc[u] = ((hw[u] & kmask) << kb) | (lw[u] & kmask);
                v0[u] = __uint_as_float(hw[u] & ~kmask);
                v1[u] = __uint_as_float(lw[u] & ~kmask);
                pend[u] = rec >= r0 && rec < r1 && loc[u] < te;
            }
            // wavefront-scope relaxed atomics: LDS accesses that complete in
            // program order for the wave (one wave per workgroup)
            auto round = [&](uint32_t u) {
                if (pend[u])
                    __hip_atomic_store(tag + loc[u], 0xffffffffu, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
                if (pend[u])
                    __hip_atomic_fetch_min(tag + loc[u], lane, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                if (pend[u] && __hip_atomic_load(tag + loc[u], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WAVEFRONT) == lane) {
                    float2 a = acc[loc[u]];
                    a.x += v0[u];
                    a.y += v1[u];
                    acc[loc[u]] = a;
                    pend[u] = false;
                }
            };
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) round(u);
            bool left = false;
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) left |= pend[u];
            while (__ballot(left)) {
#pragma unroll
                for (uint32_t u = 0; u < kPer; ++u)
                    if (__ballot(pend[u])) round(u);
                left = false;
#pragma unroll
                for (uint32_t u = 0; u < kPer; ++u) left |= pend[u];
            }
        }
        const uint32_t ne = (n_entries - tbase) < te ? (n_entries - tbase) : te;
        if (owner) {
            for (uint32_t i = lane; i < ne; i += 64) {
                const float2 a = acc[i];
                if (a.x != 0.f || a.y != 0.f) {
                    const float2 d = dtable[tbase + i];
                    dtable[tbase + i] = make_float2(d.x + a.x, d.y + a.y);
                }
            }
        } else {
            float2 *slab = partial + (size_t)it * te;
            for (uint32_t i = lane; i < ne; i += 64) slab[i] = acc[i];
        }
    }
}

__global__ void __launch_bounds__(64)
det_accum(int tb, int n_tiles, uint32_t n_entries, const uint32_t *__restrict__ start,
          const uint32_t *__restrict__ item_start, const uint32_t *__restrict__ n_items,
          const uint2 *__restrict__ recs, float2 *__restrict__ dtable,
          float2 *__restrict__ partial, uint32_t item) {
    extern __shared__ float2 acc[];                                   // [te] sums
    const uint32_t te = 1u << tb;
    uint2 *win = reinterpret_cast<uint2 *>(acc + te);                // [512] staged records
    const uint32_t lane = threadIdx.x;
    const uint32_t items = *n_items;
    const int kb = (tb + 1) >> 1;
    const uint32_t kmask = (1u << kb) - 1u;
    constexpr uint32_t kPer = 8, kWin = 64u * kPer;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        int lo = 0, hi = n_tiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_start[mid] <= it) lo = mid;
            else hi = mid - 1;
        }
        const int t = lo;
        const uint32_t first = it - item_start[t];
        const uint32_t r0 = start[t] + first * item;
        const uint32_t r1e = r0 + item;
        const uint32_t r1 = r1e < start[t + 1] ? r1e : start[t + 1];
        const bool owner = (item_start[t + 1] - item_start[t]) == 1u;
        for (uint32_t i = lane; i < te; i += 64) acc[i] = make_float2(0.f, 0.f);
        const uint32_t tbase = (uint32_t)t << tb;
        for (uint32_t base = r0 & ~(kPer - 1u); base < r1; base += kWin) {
            __syncthreads();
            const uint4 *q = reinterpret_cast<const uint4 *>(recs + base + lane * kPer);
            uint4 *wq = reinterpret_cast<uint4 *>(win + lane * kPer);
#pragma unroll
            for (int j = 0; j < 4; ++j) wq[j] = q[j];
            __syncthreads();
            const uint32_t u0 = r0 > base ? r0 - base : 0u;
            const uint32_t u1 = r1 - base < kWin ? r1 - base : kWin;
            for (uint32_t u = u0; u < u1; ++u) {
                const uint2 r = win[u];
                const uint32_t loc = ((r.x & kmask) << kb) | (r.y & kmask);
                if ((loc & 63u) == lane && loc < te) {
                    atomicAdd(&acc[loc].x, __uint_as_float(r.x & ~kmask));
                    atomicAdd(&acc[loc].y, __uint_as_float(r.y & ~kmask));
                }
            }
        }
        __syncthreads();
        const uint32_t ne = (n_entries - tbase) < te ? (n_entries - tbase) : te;
        if (owner) {
            for (uint32_t i = lane; i < ne; i += 64) {
                const float2 a = acc[i];
                if (a.x != 0.f || a.y != 0.f) {
                    const float2 d = dtable[tbase + i];
                    dtable[tbase + i] = make_float2(d.x + a.x, d.y + a.y);
                }
            }
        } else {
            float2 *slab = partial + (size_t)it * te;
            for (uint32_t i = lane; i < ne; i += 64) slab[i] = acc[i];
        }
        __syncthreads();
    }
}

nvr_status launch_scatter_det(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                              const float *x, const void *table, const float *dfeat,
                              float *dtable, float *dx_parts, void *ws, hipStream_t st,
                              const uint32_t *jac) {
    if (cap <= 0) return NVR_OK;
    NVR_TRY(scatter_check(p));
    const int tb = tile_bits(p);
    const int nt = scatter_tiles(p);
    const int lt = level_tiles(p, tb);
    const DetSeg sg = det_segments(p, tb);
    ScatterWs w = carve_scatter(p, ws, cap);
    uint32_t *seg = (uint32_t *)((char *)ws + ((scatter_ws_bytes(p, cap) + 255) & ~size_t(255)));
    const uint32_t n_records = (uint32_t)((uint64_t)cap * p.L * 8 < 0xffffffffull
                                              ? (uint64_t)cap * p.L * 8 : 0xffffffffull);
    const int lpg = (p.L + kXcds - 1) / kXcds;
    const unsigned gr = grid_for(cap, kDetBlock, 512) * kXcds;
    int dev = 0;
    NVR_HIP(hipGetDevice(&dev));
    static std::atomic<uint64_t> det_lds_ok{0};
    const uint64_t dev_bit = 1ull << (dev & 63);
    if (!(det_lds_ok.load() & dev_bit)) {
        const int most = (int)det_lds_bytes(kMaxLevelTiles);
        const void *fns[] = {(const void *)det_emit<1>, (const void *)det_emit<2>,
                             (const void *)det_emit<3>, (const void *)det_emit<4>};
        for (const void *f : fns)
            NVR_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, most));
        NVR_HIP(hipFuncSetAttribute((const void *)det_accum,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)((sizeof(float2) << kMaxTileBits) + sizeof(uint2) * 512)));
        NVR_HIP(hipFuncSetAttribute((const void *)det_accum_min,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)((sizeof(float2) + sizeof(uint32_t)) * kDetFastEntries)));
        det_lds_ok.fetch_or(dev_bit);
    }
    zero_u32<<<grid_for(nt + 1, 256, 64), 256, 0, st>>>(w.count, nt + 1);
    NVR_LAUNCHED();
    const size_t clds = sizeof(uint32_t) * lt;
    switch (lpg) {
    case 1: det_count<1><<<gr, kDetBlock, clds, st>>>(p, tb, sg, n, n_dev, cap, x, seg, w.count); break;
    case 2: det_count<2><<<gr, kDetBlock, clds, st>>>(p, tb, sg, n, n_dev, cap, x, seg, w.count); break;
    case 3: det_count<3><<<gr, kDetBlock, clds, st>>>(p, tb, sg, n, n_dev, cap, x, seg, w.count); break;
    default: det_count<4><<<gr, kDetBlock, clds, st>>>(p, tb, sg, n, n_dev, cap, x, seg, w.count); break;
    }
    NVR_LAUNCHED();
    scatter_scan<<<1, 1024, 0, st>>>(nt, w.count, w.start, w.cursor, w.item_start, w.n_items,
                                     item_records(cap, p.L));
    NVR_LAUNCHED();
    {
        const int S = sg.at[p.L];
        const int64_t ncap = (cap + kDetBlock - 1) / kDetBlock;
        uint32_t *psum = seg + (size_t)ncap * S;
        uint32_t *pbase = psum + (size_t)kSegParts * S;
        const unsigned gs = (unsigned)(((int64_t)S * kSegParts + 255) / 256);
        det_seg_sums<<<gs, 256, 0, st>>>(sg, p.L, n, n_dev, cap, seg, psum);
        NVR_LAUNCHED();
        det_seg_bases<<<(nt + 255) / 256, 256, 0, st>>>(p, tb, sg, nt, w.start, psum, pbase);
        NVR_LAUNCHED();
        det_seg_apply<<<gs, 256, 0, st>>>(sg, p.L, n, n_dev, cap, pbase, seg);
        NVR_LAUNCHED();
    }
    const size_t elds = det_lds_bytes(lt);
    const uint32_t *tab = (const uint32_t *)table;
    switch (lpg) {
    case 1: det_emit<1><<<gr, kDetBlock, elds, st>>>(p, tb, lt, sg, n, n_dev, cap, x, tab, dfeat, n_records, seg, w.rec, dx_parts, jac); break;
    case 2: det_emit<2><<<gr, kDetBlock, elds, st>>>(p, tb, lt, sg, n, n_dev, cap, x, tab, dfeat, n_records, seg, w.rec, dx_parts, jac); break;
    case 3: det_emit<3><<<gr, kDetBlock, elds, st>>>(p, tb, lt, sg, n, n_dev, cap, x, tab, dfeat, n_records, seg, w.rec, dx_parts, jac); break;
    default: det_emit<4><<<gr, kDetBlock, elds, st>>>(p, tb, lt, sg, n, n_dev, cap, x, tab, dfeat, n_records, seg, w.rec, dx_parts, jac); break;
    }
    NVR_LAUNCHED();
    if (dtable == nullptr) return NVR_OK;
    const int64_t max_items = max_items_of(cap, p.L, nt);
    const unsigned ga = (unsigned)(max_items < 65535 ? max_items : 65535);
    if ((1u << tb) <= kDetFastEntries) {
        const size_t alds = (sizeof(float2) + sizeof(uint32_t)) << tb;
        det_accum_min<<<ga, 64, alds, st>>>(tb, nt, p.off[p.L], w.start, w.item_start, w.n_items,
                                            w.rec, (float2 *)dtable, w.partial,
                                            item_records(cap, p.L));
    } else {
        const size_t alds = (sizeof(float2) << tb) + sizeof(uint2) * 512;
        det_accum<<<ga, 64, alds, st>>>(tb, nt, p.off[p.L], w.start, w.item_start, w.n_items,
                                        w.rec, (float2 *)dtable, w.partial, item_records(cap, p.L));
    }
    NVR_LAUNCHED();
    scatter_reduce<<<dim3(((1u << tb) + 255) / 256, nt), 256, 0, st>>>(
        tb, p.off[p.L], w.item_start, w.partial, (float2 *)dtable);
    NVR_LAUNCHED();
    return NVR_OK;
}

// Row-major feature gradients dfeat[n][2L] to the level-group-planar layout
// emit reads, [8][n][2 lpg] (level l = g + 8 m at [g][s][2m, 2m+1]; slots of
// levels >= L hold 0).  Each workgroup pass moves 128 whole rows through LDS,
// so both the reads and the eight per-group writes are contiguous runs.
constexpr int kPlanarRows = 128;

__global__ void __launch_bounds__(256)
scatter_planarize(int L, int lpg, int64_t n, const float *__restrict__ dfeat,
                  float *__restrict__ out, const int32_t *__restrict__ n_dev = nullptr,
                  int64_t cap = 0) {
    extern __shared__ float rows[];                    // [kPlanarRows][2L + 1]
    const int w = 2 * L, wp = w + 1, q = 2 * lpg;
    const int64_t stride = n_dev ? cap : n;           // planes are [cap][q] with a device count
    if (n_dev) n = count_of(n, n_dev, cap);
    for (int64_t s0 = (int64_t)blockIdx.x * kPlanarRows; s0 < n;
         s0 += (int64_t)gridDim.x * kPlanarRows) {
        const int ns = (int)(n - s0 < kPlanarRows ? n - s0 : kPlanarRows);
        const float *src = dfeat + (size_t)s0 * w;
        for (int i = threadIdx.x; i < ns * w; i += blockDim.x) rows[(i / w) * wp + i % w] = src[i];
        __syncthreads();
        for (int g = 0; g < kXcds; ++g) {
            float *dst = out + ((size_t)g * stride + s0) * q;
            for (int j = threadIdx.x; j < ns * q; j += blockDim.x) {
                const int r = j / q, c = j % q, l = g + kXcds * (c >> 1);
                dst[j] = l < L ? rows[r * wp + 2 * l + (c & 1)] : 0.f;
            }
        }
        __syncthreads();
    }
}

// dx[n][3] += the eight level groups' partial position gradients [8][n][3].
__global__ void __launch_bounds__(256)
scatter_dx_sum(int64_t n3, const float *__restrict__ parts, float *__restrict__ dx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        float a = 0.f;
#pragma unroll
        for (int g = 0; g < kXcds; ++g) a += parts[(size_t)g * n3 + i];
        dx[i] += a;
    }
}

// Bytes of the public entry point's workspace: the binned scatter's, then the
// planar feature gradients [8][n][2 lpg] and the partial position gradients
// [8][n][3].
static size_t public_ws_bytes(const GridParams &p, int64_t n, size_t *planar_at, size_t *parts_at,
                              bool det = false) {
    const int lpg = (p.L + kXcds - 1) / kXcds;
    size_t b = ((det ? scatter_det_ws_bytes(p, n) : scatter_ws_bytes(p, n)) + 255) & ~size_t(255);
    *planar_at = b;
    b += sizeof(float) * (size_t)kXcds * n * 2 * lpg;
    b = (b + 255) & ~size_t(255);
    *parts_at = b;
    b += sizeof(float) * (size_t)kXcds * n * 3;
    return b;
}

nvr_status launch_scatter_emit_only(const GridParams &p, int64_t n, const int32_t *n_dev,
                                    int64_t cap, const float *x, const void *table,
                                    const float *dfeat, void *ws, hipStream_t st,
                                    int emit_chunks, int emit_block) {
    return launch_scatter(p, n, n_dev, cap, x, table, dfeat, nullptr, nullptr, ws, st,
                          /*counted=*/true, emit_chunks, emit_block);
}

// Table gradient of row-major feature gradients dfeat[cap][2L] over the first
// count_of(n, n_dev, cap) samples: regrouped into the level-group planes, then
// the binned scatter (det: its deterministic variant).  ws:
// scatter_rows_ws_bytes(p, cap, det) bytes.
size_t scatter_rows_ws_bytes(const GridParams &p, int64_t cap, bool det) {
    const int lpg = (p.L + kXcds - 1) / kXcds;
    const size_t sc = det ? scatter_det_ws_bytes(p, cap) : scatter_ws_bytes(p, cap);
    return ((sc + 255) & ~size_t(255)) + sizeof(float) * (size_t)kXcds * cap * 2 * lpg;
}

nvr_status launch_scatter_rows(const GridParams &p, int64_t n, const int32_t *n_dev, int64_t cap,
                               const float *x, const float *dfeat, float *dtable, void *ws,
                               hipStream_t st, bool det) {
    if (cap <= 0) return NVR_OK;
    const int lpg = (p.L + kXcds - 1) / kXcds;
    const size_t sc = det ? scatter_det_ws_bytes(p, cap) : scatter_ws_bytes(p, cap);
    float *planar = (float *)((char *)ws + ((sc + 255) & ~size_t(255)));
    scatter_planarize<<<grid_for(cap, kPlanarRows, 8192), 256,
                        sizeof(float) * kPlanarRows * (2 * p.L + 1), st>>>(p.L, lpg, n, dfeat,
                                                                           planar, n_dev, cap);
    NVR_LAUNCHED();
    if (det)
        return launch_scatter_det(p, n, n_dev, cap, x, nullptr, planar, dtable, nullptr, ws, st);
    return launch_scatter(p, n, n_dev, cap, x, nullptr, planar, dtable, nullptr, ws, st,
                          /*counted=*/false, 1024, 512);
}

}  // namespace nvr

using namespace nvr;

extern "C" size_t nvr_encode_bwd_workspace(const nvr_grid_desc *g, int64_t n) {
    if (check_grid(g) != NVR_OK || n < 0) return 0;
    size_t planar_at, parts_at;
    return public_ws_bytes(make_grid_params(g), n, &planar_at, &parts_at);
}

extern "C" size_t nvr_encode_bwd_deterministic_workspace(const nvr_grid_desc *g, int64_t n) {
    if (check_grid(g) != NVR_OK || n < 0) return 0;
    size_t planar_at, parts_at;
    return public_ws_bytes(make_grid_params(g), n, &planar_at, &parts_at, true);
}

// The public binned entry points: dfeat row-major [n][2L] (regrouped first)
// or already level-group planar [8][n][2 lpg]; det selects the deterministic
// variant.
static nvr_status binned_public(const nvr_grid_desc *g, int64_t n, const float *x,
                                const void *table, const float *dfeat, bool grouped,
                                float *dtable, float *dx, void *workspace, nvr_stream stream,
                                bool det = false) {
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
    const hipStream_t st = hs(stream);
    size_t planar_at, parts_at;
    public_ws_bytes(p, n, &planar_at, &parts_at, det);
    const float *planar = dfeat;
    float *parts = dx ? (float *)((char *)workspace + parts_at) : nullptr;
    if (!grouped) {
        float *buf = (float *)((char *)workspace + planar_at);
        const int lpg = (p.L + kXcds - 1) / kXcds;
        scatter_planarize<<<grid_for(n, kPlanarRows, 8192), 256,
                            sizeof(float) * kPlanarRows * (2 * p.L + 1), st>>>(p.L, lpg, n, dfeat,
                                                                               buf);
        NVR_LAUNCHED();
        planar = buf;
    }
    // 512-sample emit chunks, 1024 chunks per level group: the shape the step's
    // tuner settles on for millions of samples
    if (det)
        NVR_TRY(launch_scatter_det(p, n, nullptr, n, x, table, planar, dtable, parts, workspace,
                                   st));
    else
        NVR_TRY(launch_scatter(p, n, nullptr, n, x, table, planar, dtable, parts, workspace, st,
                               /*counted=*/false, 1024, 512));
    if (dx) {
        scatter_dx_sum<<<grid_for(3 * n, 256, 8192), 256, 0, st>>>(3 * n, parts, dx);
        NVR_LAUNCHED();
    }
    return NVR_OK;
}

extern "C" nvr_status nvr_encode_bwd_binned(const nvr_grid_desc *g, int64_t n, const float *x,
                                            const void *table, const float *dfeat, float *dtable,
                                            float *dx, void *workspace, nvr_stream stream) {
    return binned_public(g, n, x, table, dfeat, false, dtable, dx, workspace, stream);
}

extern "C" nvr_status nvr_encode_bwd_binned_grouped(const nvr_grid_desc *g, int64_t n,
                                                    const float *x, const void *table,
                                                    const float *dfeat, float *dtable, float *dx,
                                                    void *workspace, nvr_stream stream) {
    return binned_public(g, n, x, table, dfeat, true, dtable, dx, workspace, stream);
}

extern "C" nvr_status nvr_encode_bwd_deterministic(const nvr_grid_desc *g, int64_t n,
                                                   const float *x, const void *table,
                                                   const float *dfeat, float *dtable, float *dx,
                                                   void *workspace, nvr_stream stream) {
    return binned_public(g, n, x, table, dfeat, false, dtable, dx, workspace, stream, true);
}
