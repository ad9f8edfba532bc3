// Occupancy-grid maintenance: the density grid behind the marcher's bitfield
// (the fields' Instant-NGP back-end, Sec. 4.3).  One update:
//   1. occ_decay   -- g <- decay * g over all cells;
//   2. the field's encode + network forward at the probe points -> sigma;
//   3. occ_max     -- g[c_i] <- max(g[c_i], sigma_i); non-negative floats order
//                     like their bit patterns, so an integer atomic max gives
//                     the same result in any order;
//   4. occ_sum / occ_tau -- mean(g) in float64, per-block partials summed in a
//                     fixed order (deterministic); tau = min(tau_max, mean);
//   5. occ_bits    -- bit c & 31 of word c >> 5 is set iff g[c] > tau.
#include "launch.hpp"

namespace nvr {
namespace {

constexpr int kOccBlock = 256;
constexpr int kOccSumBlocks = 1024;

__global__ void __launch_bounds__(kOccBlock)
occ_decay(int64_t n, float decay, float *__restrict__ g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        g[i] = g[i] * decay;
}

__global__ void __launch_bounds__(kOccBlock)
occ_max(int64_t m, int64_t n_cells, const int32_t *__restrict__ cells,
        const float *__restrict__ sigma, float *__restrict__ g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = cells[i];
        const float s = sigma[i];
        if (c >= 0 && c < n_cells && s > 0.f)   // cells outside the grid are ignored
            atomicMax(reinterpret_cast<unsigned int *>(g + c), __float_as_uint(s));
    }
}

__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kOccBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(kOccBlock)
occ_sum(int64_t n, const float *__restrict__ g, double *__restrict__ partial) {
    __shared__ double red[kOccBlock];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += (double)g[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kOccBlock)
occ_tau(int nb, const double *__restrict__ partial, int64_t n, float tau_max,
        float *__restrict__ tau) {
    __shared__ double red[kOccBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) {
        const float mean = (float)(t / (double)n);
        *tau = mean < tau_max ? mean : tau_max;
    }
}

__global__ void __launch_bounds__(kOccBlock)
occ_bits(int64_t n_words, int64_t n_cells, const float *__restrict__ g,
         const float *__restrict__ tau, uint32_t *__restrict__ bits) {
    const float t = *tau;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n_words;
         w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0u;
        for (int j = 0; j < 32; ++j) {
            const int64_t c = 32 * w + j;
            if (c < n_cells && g[c] > t) v |= 1u << j;
        }
        bits[w] = v;
    }
}

struct OccWs {
    void *feat;
    float *sigma, *rgb, *mlp;
    double *partial;
};

size_t occ_ws(const Net &net, int precision, int64_t m, OccWs *w, void *base) {
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const bool bf = precision == NVR_BF16;
    const size_t sz[5] = {
        bf ? sizeof(uint16_t) * 32 * (size_t)m : sizeof(float) * net.n_in * (size_t)m,  // feat
        sizeof(float) * (size_t)m,                                                      // sigma
        sizeof(float) * 3 * (size_t)m,                                                  // rgb
        bf ? 0 : plain_workspace(net, m),                                               // mlp
        sizeof(double) * kOccSumBlocks,                                                 // partial
    };
    size_t off[5], b = 0;
    for (int i = 0; i < 5; ++i) {
        off[i] = b;
        b += up(sz[i]);
    }
    if (w) {
        char *p = (char *)base;
        w->feat = sz[0] ? p + off[0] : nullptr;
        w->sigma = (float *)(p + off[1]);
        w->rgb = (float *)(p + off[2]);
        w->mlp = sz[3] ? (float *)(p + off[3]) : nullptr;
        w->partial = (double *)(p + off[4]);
    }
    return b;
}

nvr_status occ_check(const nvr_field *f, int precision, int64_t m, Net *net) {
    NVR_REQUIRE(f != nullptr, NVR_EINVAL, "field is NULL");
    NVR_TRY(check_grid(&f->grid));
    NVR_TRY(build_net(&f->mlp, net));
    NVR_REQUIRE(net->n_in == f->grid.n_levels * f->grid.n_features, NVR_EINVAL,
                "network input width %d != encoding width %d", net->n_in,
                f->grid.n_levels * f->grid.n_features);
    NVR_REQUIRE(!f->has_warp, NVR_EUNSUPPORTED,
                "occupancy upkeep of a warped field needs the live-space density");
    NVR_REQUIRE(f->march.occ_res >= 1 && f->march.occ_res <= 1024, NVR_EINVAL,
                "occ_res out of 1..1024");
    NVR_REQUIRE(m >= 0 && m < (1ll << 31), NVR_EINVAL, "m out of range");
    NVR_REQUIRE(precision == NVR_F32 || precision == NVR_BF16, NVR_EINVAL,
                "precision must be F32 or BF16");
    if (precision == NVR_BF16) {
        NVR_REQUIRE(f->grid.n_levels == 16, NVR_EUNSUPPORTED,
                    "the bf16 path uses the planar 16-level layout");
        NVR_TRY(mfma_check(*net));
    }
    return NVR_OK;
}

}  // namespace
}  // namespace nvr

using namespace nvr;

extern "C" size_t nvr_occupancy_workspace(const nvr_field *f, int32_t precision, int64_t m) {
    Net net;
    if (occ_check(f, precision, m, &net) != NVR_OK) return 0;
    return occ_ws(net, precision, m, nullptr, nullptr);
}

extern "C" nvr_status nvr_occupancy_update(const nvr_field *f, int32_t precision, int64_t m,
                                           const int32_t *cells, const float *points, float decay,
                                           float tau_max, float *grid, uint32_t *bits, float *tau,
                                           void *workspace, nvr_stream stream) {
    clear_error();
    Net net;
    NVR_TRY(occ_check(f, precision, m, &net));
    NVR_REQUIRE(decay >= 0.f && decay <= 1.f, NVR_EINVAL, "decay out of [0, 1]");
    NVR_REQUIRE(tau_max > 0.f, NVR_EINVAL, "tau_max must be positive");
    NVR_REQUIRE(grid && bits && tau && workspace, NVR_EINVAL, "NULL array");
    NVR_REQUIRE(m == 0 || (cells && points), NVR_EINVAL, "NULL probes");
    NVR_REQUIRE(aligned(grid, 4) && aligned(bits, 4) && aligned(tau, 4) && aligned(cells, 4) &&
                    aligned(points, 4) && aligned(workspace, 256),
                NVR_EINVAL, "misaligned array");
    if (m > 0) {
        if (precision == NVR_BF16)
            NVR_REQUIRE(f->table_half && f->params, NVR_EINVAL, "NULL fp16 table or params");
        else
            NVR_REQUIRE(f->table && f->params, NVR_EINVAL, "NULL table or params");
    }
    const hipStream_t st = hs(stream);
    const int64_t res = f->march.occ_res;
    const int64_t n_cells = res * res * res;
    const int64_t n_words = (n_cells + 31) / 32;
    OccWs w;
    occ_ws(net, precision, m, &w, workspace);
    occ_decay<<<grid_for(n_cells, kOccBlock, 8192), kOccBlock, 0, st>>>(n_cells, decay, grid);
    NVR_LAUNCHED();
    if (m > 0) {
        // the probes' density: the training step's encode and network forward
        // (the direction input is unused by sigma; the points serve as one)
        const GridParams gp = make_grid_params(&f->grid);
        if (precision == NVR_BF16) {
            NVR_TRY(launch_encode_fwd(gp, m, nullptr, m, points, f->table_half, NVR_F16, w.feat,
                                      NVR_F16, true, st));
            NVR_TRY(mfma_fwd(net, m, nullptr, m, (const uint16_t *)w.feat, true, points, nullptr,
                             f->params, true, w.sigma, w.rgb, st));
        } else {
            NVR_TRY(launch_encode_fwd(gp, m, nullptr, m, points, f->table, NVR_F32, w.feat,
                                      NVR_F32, false, st));
            PlainView F{(float *)w.feat, 1, net.n_in};
            NVR_TRY(plain_fwd(net, m, nullptr, m, F, points, nullptr, f->params, w.sigma, w.rgb,
                              w.mlp, st));
        }
        occ_max<<<grid_for(m, kOccBlock, 8192), kOccBlock, 0, st>>>(m, n_cells, cells, w.sigma,
                                                                   grid);
        NVR_LAUNCHED();
    }
    occ_sum<<<kOccSumBlocks, kOccBlock, 0, st>>>(n_cells, grid, w.partial);
    NVR_LAUNCHED();
    occ_tau<<<1, kOccBlock, 0, st>>>(kOccSumBlocks, w.partial, n_cells, tau_max, tau);
    NVR_LAUNCHED();
    occ_bits<<<grid_for(n_words, kOccBlock, 8192), kOccBlock, 0, st>>>(n_words, n_cells, grid,
                                                                      tau, bits);
    NVR_LAUNCHED();
    return NVR_OK;
}
