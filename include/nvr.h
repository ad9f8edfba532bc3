/*
 * nvr.h -- C ABI of the MI355X (gfx950) hot path of Instant-NVR's on-the-fly
 * radiance-field back-end: march rays with occupancy skipping, warp live human
 * samples into the canonical space, encode with a multiresolution hash grid,
 * evaluate the density and colour networks, alpha-composite, back-propagate the
 * colour / depth loss and update the parameters with Adam.
 *
 * Paper: "Instant-NVR: Instant Neural Volumetric Rendering for Human-object
 * Interactions from Monocular RGBD Stream" (CVPR 2023).  Each entry point
 * below names the passage that defines what it computes.
 *
 * Conventions (every entry point):
 *   - Array pointers are DEVICE pointers owned by the caller unless a comment
 *     says "host".  Descriptors (structs) are host memory, read during the call.
 *   - Arrays are dense, row-major, naturally aligned; float32 unless stated.
 *     "(acc)" outputs are ACCUMULATED into (the caller zeroes them); others are
 *     overwritten.  "nullable" arguments may be NULL to skip that output/input.
 *   - All work is enqueued on `stream` (0 = the null stream); nothing
 *     synchronises implicitly unless a comment says so.
 *   - Shapes and descriptors are validated on the host BEFORE anything is
 *     launched; on failure the call returns a negative nvr_status, launches
 *     nothing and sets a thread-local message readable by nvr_last_error().
 *     No entry point aborts or exits.
 *   - Sample counts that are only known on the device (after marching) are
 *     passed as `const int32_t *n_dev`: kernels read the count there and are
 *     launched for `capacity` samples, so no host synchronisation is needed.
 */
#ifndef NVR_H
#define NVR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *nvr_stream;   /* hipStream_t */

typedef enum {
    NVR_OK = 0,
    NVR_EINVAL = -1,        /* bad descriptor, size, pointer or alignment */
    NVR_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. F != 2) */
    NVR_EHIP = -3,          /* a HIP runtime call failed */
    NVR_ENOMEM = -4,        /* device allocation failed (context workspace) */
    NVR_ENONFINITE = -5,    /* non-finite gradients: step skipped (informational) */
    NVR_EOVERFLOW = -6      /* more samples than the given capacity */
} nvr_status;

typedef enum { NVR_F32 = 0, NVR_F16 = 1, NVR_BF16 = 2 } nvr_dtype;

/* Message of the last failing call on this thread ("" if none). */
const char *nvr_last_error(void);
/* Library version string. */
const char *nvr_version(void);

/* ------------------------------------------------------------------------
 * Multiresolution hash grid.  The paper extracts per-point features from a
 * hash table for each field (Sec. 4.2, "Separated instant neural
 * representation"), delegating the encoding to Instant-NGP: level l has
 * resolution N_l = floor(N_min * b^l), b = exp((ln N_max - ln N_min)/(L-1))
 * (float64 on the host); x_hat = clamp((x - aabb_min)/(aabb_max - aabb_min),
 * 0, 1); x_l = x_hat * N_l; cell c = min(floor(x_l), N_l - 1); trilinear
 * weights over the 8 corners; a level with (N_l+1)^3 <= T vertices is
 * indexed densely (cx + (N_l+1)(cy + (N_l+1) cz)), else by
 * (cx*1 ^ cy*2654435761 ^ cz*805459861) mod 2^32 & (T-1).
 * Table layout: [n_entries][F] with level l at entries offset[l]..offset[l+1);
 * each level's slice is its vertex count rounded up to a multiple of 8 entries
 * (the padding entries are never read or written by the encoding, and the
 * aligned slices let the gather fetch x-neighbouring corners together).
 * ---------------------------------------------------------------------- */
#define NVR_MAX_LEVELS 32
typedef struct {
    int32_t n_levels;            /* L, 1..32 */
    int32_t n_features;          /* F, must be 2 */
    int32_t log2_table;          /* log2 T, 4..24 */
    int32_t res[NVR_MAX_LEVELS];     /* N_l */
    int32_t dense[NVR_MAX_LEVELS];   /* 1 if level l is dense */
    int64_t offset[NVR_MAX_LEVELS + 1];  /* entry offsets; offset[L] = n_entries */
    float aabb_min[3], aabb_max[3];
} nvr_grid_desc;

/* Fill `g` (host) from the level ladder parameters.  aabb_* are host arrays. */
nvr_status nvr_grid_init(nvr_grid_desc *g, int32_t n_levels, int32_t n_features,
                         int32_t log2_table, int32_t res_min, int32_t res_max,
                         const float *aabb_min, const float *aabb_max);

/* feat[n][L*F] = encoding of x[n][3] (world positions).  table_dtype is
 * NVR_F32 or NVR_F16; feat_dtype NVR_F32, NVR_F16 or NVR_BF16.  The fp16-table
 * path is the level-split kernel (each XCD serves a fixed subset of levels). */
nvr_status nvr_encode_fwd(const nvr_grid_desc *g, int64_t n, const float *x,
                          const void *table, nvr_dtype table_dtype,
                          void *feat, nvr_dtype feat_dtype, nvr_stream stream);

/* Backward: dtable[e][f] += sum over samples/corners of w * dfeat (acc, f32);
 * dx[n][3] += d/dx of sum(feat * dfeat) (acc, nullable; 0 where x_hat was
 * clamped).  dfeat is [n][L*F] float32. */
nvr_status nvr_encode_bwd(const nvr_grid_desc *g, int64_t n, const float *x,
                          const void *table, nvr_dtype table_dtype,
                          const float *dfeat, float *dtable, float *dx,
                          nvr_stream stream);

/* Same gradients as nvr_encode_bwd for a float16 table, without a global
 * atomic per contribution: dfeat is first regrouped by level group (the eight
 * XCDs each serve a fixed subset of levels), the contributions are binned by
 * table tiles of 2^10..2^14 entries (count, scan, append) and each tile is
 * summed in LDS and added into dtable once; dx (nullable) receives the sum of
 * the level groups' position gradients.  dtable must be 8-byte aligned;
 * workspace (device, 256-byte aligned) of nvr_encode_bwd_workspace(g, n)
 * bytes, owned by the caller, is overwritten.  Unsupported ladders (more than
 * 8192 tiles, a level over 2048 tiles, more than 32 levels) return
 * NVR_EUNSUPPORTED. */
size_t nvr_encode_bwd_workspace(const nvr_grid_desc *g, int64_t n);
nvr_status nvr_encode_bwd_binned(const nvr_grid_desc *g, int64_t n, const float *x,
                                 const void *table, const float *dfeat, float *dtable,
                                 float *dx, void *workspace, nvr_stream stream);

/* nvr_encode_bwd_binned with every sum formed in an order fixed by the inputs
 * alone, so repeated calls give bit-identical dtable and dx whatever the
 * timing of the launch: each tile's records are placed by level, then by
 * chunk of 512 samples, wavefront, corner and lane (counts per chunk and
 * tile are formed and scanned first, instead of reserving ranges with
 * atomics), and one lane adds all records of an entry in that order.  Same
 * arguments, record rounding and errors as nvr_encode_bwd_binned; workspace
 * (device, 256-byte aligned) of nvr_encode_bwd_deterministic_workspace(g, n)
 * bytes (it adds one uint32 per chunk and tile), owned by the caller. */
size_t nvr_encode_bwd_deterministic_workspace(const nvr_grid_desc *g, int64_t n);
nvr_status nvr_encode_bwd_deterministic(const nvr_grid_desc *g, int64_t n, const float *x,
                                        const void *table, const float *dfeat, float *dtable,
                                        float *dx, void *workspace, nvr_stream stream);

/* The level-group ("grouped") layout the fused step keeps features and their
 * gradients in: [8][n][2 lpg] with lpg = ceil(L / 8), level l = g + 8 m at
 * [g][s][2m, 2m+1] (slots of levels >= L are written as 0 / ignored); F = 2
 * only.  Each XCD serves one plane, so neither call regroups anything.
 * nvr_encode_fwd_grouped: fp16 table, fp16 features (same values as
 * nvr_encode_fwd with table_dtype = feat_dtype = NVR_F16).
 * nvr_encode_bwd_binned_grouped: nvr_encode_bwd_binned with dfeat (float32)
 * in the grouped layout; same workspace and errors. */
nvr_status nvr_encode_fwd_grouped(const nvr_grid_desc *g, int64_t n, const float *x,
                                  const void *table, void *feat, nvr_stream stream);
nvr_status nvr_encode_bwd_binned_grouped(const nvr_grid_desc *g, int64_t n, const float *x,
                                         const void *table, const float *dfeat,
                                         float *dtable, float *dx, void *workspace,
                                         nvr_stream stream);

/* ------------------------------------------------------------------------
 * Ray marching with occupancy skipping (the back-end is built on Instant-NGP,
 * Sec. 4.3; its marcher is not described in the paper).  Per ray: clip
 * o + t d to the box (slab method) intersected with [near, far]; samples at
 * t_i = t_n + (i + 1/2) * step while t_i < t_f, at most max_steps; keep a
 * sample iff its occupancy voxel's bit is set (voxel v = clamp(floor((x -
 * aabb_min) * (occ_res/side)), 0, occ_res-1), index vx + R(vy + R vz), bit
 * idx&31 of word idx>>5).  These integer decisions are taken in IEEE float32,
 * one rounding per operation, no fused multiply-add.
 * ---------------------------------------------------------------------- */
typedef struct {
    float aabb_min[3], aabb_max[3];
    float near_t, far_t;
    float step;                  /* <= 0: float(sqrt(3) * max side / max_steps) */
    int32_t max_steps;           /* 1..1024 */
    int32_t occ_res;             /* 0: keep every sample */
} nvr_march_desc;

/* Bytes of scratch nvr_march needs for n_rays rays. */
size_t nvr_march_workspace(int64_t n_rays);

/* Marches rays [ray_begin, ray_end) of o[n_rays][3], d[n_rays][3]; rays outside
 * the range get no samples.  Writes off[n_rays+1] (ray r owns samples
 * off[r]..off[r+1]-1, ray-major, increasing t), and for each sample ray_id, t,
 * dt and its position x[3]; n_dev[0] = total kept samples (may exceed
 * capacity: samples past capacity are not written, and the caller must treat
 * n_dev[0] > capacity as NVR_EOVERFLOW).  occ is the bitfield (nullable iff
 * occ_res == 0).  workspace: nvr_march_workspace(n_rays) bytes. */
nvr_status nvr_march(const nvr_march_desc *m, int64_t n_rays, int64_t ray_begin,
                     int64_t ray_end, const float *o, const float *d,
                     const uint32_t *occ, int64_t capacity, int32_t *off,
                     int32_t *ray_id, float *t, float *dt, float *x, int32_t *n_dev,
                     void *workspace, nvr_stream stream);

/* nvr_march without a workspace argument and without any device allocation,
 * for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, outputs
 * and errors as nvr_march; the scan's block sums live in a fixed library array
 * of 256 KiB per device (one int32 per 256 rays), so n_rays is limited to
 * 2^24 (larger counts return NVR_EINVAL before any launch).  That array's
 * device address is looked up on the first call made with a device current
 * (the stream, if not the null stream, must belong to the current device);
 * every call on one device shares it, so calls that overlap in time on one
 * device (different streams, threads) race and must be serialised by the
 * caller.  Each call rewrites every entry it reads, so nothing carries over
 * from the previous call. */
nvr_status nvr_march_noalloc(const nvr_march_desc *m, int64_t n_rays, int64_t ray_begin,
                             int64_t ray_end, const float *o, const float *d,
                             const uint32_t *occ, int64_t capacity, int32_t *off,
                             int32_t *ray_id, float *t, float *dt, float *x, int32_t *n_dev,
                             nvr_stream stream);

/* ------------------------------------------------------------------------
 * Hybrid warp live -> canonical (Sec. 4.2, Eq. 4, with the node weight of
 * Sec. 4.1 after Eq. 1, r = 0.1, and the voxel look-up of neighbour nodes of
 * "On-the-fly Radiance Fields").  Per sample x (live): inverse skinning over
 * the k_joints nearest joints (Gaussian weights, sigma_skin, normalised;
 * y = sum_j w_j (R_j x + t_j) with bones given as live->canonical [R|t]), then
 * the inverse node blend over the k_nodes ids listed for x's live voxel:
 * b = sum_i s_i w_i conj(dq_i), w_i = exp(-(|y-g_i|^2 - min_k|y-g_k|^2)/r^2),
 * s_i = sign <q_r,i, q_r,first>, c = b/|b_r|, z = R(c_r) y + 2 vec(c_d c_r*).
 * Voxel choice, joint choice and sign are float32 decisions (see nvr_march).
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_joints;            /* <= 64 */
    int32_t k_joints;            /* 1..8 */
    float sigma_skin;            /* skinning Gaussian width (0.1) */
    int32_t n_nodes;             /* <= 65536 (uint16 ids) */
    int32_t k_nodes;             /* 1..16 */
    int32_t n_frames;            /* >= 1 */
    float r_node;                /* node influence radius r (0.1) */
    int32_t lut_res;             /* look-up grid resolution */
    float lut_min[3], lut_max[3];
} nvr_warp_desc;

typedef struct {                 /* device pointers */
    const float *joints;         /* [n_joints][3] */
    const float *bones;          /* [n_frames][n_joints][3][4] */
    const float *node_dq;        /* [n_frames][n_nodes][8] real(w,x,y,z), dual(w,x,y,z) */
    const float *node_pos;       /* [n_frames][n_nodes][3] deformed node positions */
    const uint16_t *lut;         /* [n_frames][lut_res^3][k_nodes] */
} nvr_warp_rig;

/* x_can[n][3] = warp of x_live[n][3]; frame (nullable) gives each sample's
 * frame (default 0).  n_dev (nullable) overrides n with a device count. */
nvr_status nvr_warp_fwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t n,
                        const int32_t *n_dev, const float *x_live, const int32_t *frame,
                        float *x_can, nvr_stream stream);

/* Backward of sum(dx_can . x_can): d_node_dq[n_frames][n_nodes][8] (acc)
 * through the blend; d_bones[n_frames][n_joints][12] (acc, nullable) through
 * y including y's effect on the node weights; dx_live[n][3] (acc, nullable)
 * through the skinning blend, its weights and the node weights (the joint and
 * voxel choices are locally constant).  dx_can may be given as n_parts
 * partial arrays of [n][3] laid out back to back, which are summed. */
nvr_status nvr_warp_bwd(const nvr_warp_desc *w, const nvr_warp_rig *rig, int64_t n,
                        const int32_t *n_dev, const float *x_live, const int32_t *frame,
                        const float *dx_can, int32_t n_parts, float *d_node_dq,
                        float *d_bones, float *dx_live, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Density + colour networks of a field (Sec. 4.2: geometry network E_g and
 * colour network E_c on the encoded features; widths from Instant-NGP):
 * bias-free linear layers with ReLU on hidden layers; density outputs o[16],
 * sigma = exp(clamp(o_0, -15, 15)); colour input [o, SH(d)] with real SH of
 * `sh_degree` bands (d^2 coefficients, standard real basis, Y_1 ~ (y, z, x));
 * rgb = sigmoid(last layer).  Parameters: one flat vector, each layer's
 * W[out][in] row-major, density layers first.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_in;                /* encoding width, 1..64 */
    int32_t n_density_hidden;    /* 1..4 */
    int32_t density_hidden[4];   /* widths, 1..64 */
    int32_t density_out;         /* 1..16 */
    int32_t sh_degree;           /* 1..4 */
    int32_t n_colour_hidden;     /* 1..4 */
    int32_t colour_hidden[4];    /* widths, 1..64 */
} nvr_mlp_desc;

/* Number of parameters (host out). */
nvr_status nvr_mlp_param_count(const nvr_mlp_desc *m, int64_t *count);

/* sigma[n], rgb[n][3] from feat[n][n_in] (feat_dtype) and the view direction
 * dirs[ray_id[i]] (ray_id nullable: dirs is per sample).  math = NVR_F32 runs
 * the plain float32 kernel (params float32).  math = NVR_F16 and NVR_BF16 run
 * the MFMA kernel (widths 64 / n_in <= 32 / density_out 16 / 16 + SH <= 32
 * only) with fp32 accumulation: NVR_F16 takes fp16 features and the float32
 * parameters (converted to fp16 fragments), NVR_BF16 bf16 features and a bf16
 * parameter copy; the forward runs in that type, every backward product in
 * bf16. */
nvr_status nvr_mlp_fwd(const nvr_mlp_desc *m, int64_t n, const int32_t *n_dev,
                       const void *feat, nvr_dtype feat_dtype, const float *dirs,
                       const int32_t *ray_id, const void *params, nvr_dtype math,
                       float *sigma, float *rgb, nvr_stream stream);

/* Backward from dsigma[n], drgb[n][3]: dparams (acc, f32, flat like params),
 * dfeat[n][n_in] (overwritten, f32, nullable).  Recomputes the forward.
 * workspace: nvr_mlp_workspace(m, math, n) bytes (NVR_F32: per-layer
 * activations and their gradients, unit-major; NVR_BF16: per-workgroup
 * partial weight gradients). */
size_t nvr_mlp_workspace(const nvr_mlp_desc *m, nvr_dtype math, int64_t n);
nvr_status nvr_mlp_bwd(const nvr_mlp_desc *m, int64_t n, const int32_t *n_dev,
                       const void *feat, nvr_dtype feat_dtype, const float *dirs,
                       const int32_t *ray_id, const void *params, nvr_dtype math,
                       const float *dsigma, const float *drgb, float *dparams,
                       float *dfeat, void *workspace, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Compositing (volume rendering of the density fields, Sec. 1 / Sec. 4.3;
 * NeRF quadrature): tau_i = sigma_i dt_i, T_i = exp(-sum_{j<i} tau_j),
 * w_i = T_i (1 - exp(-tau_i)); C = sum w_i c_i, D = sum w_i t_i, TN = T_n.
 * A second sample list (b, nullable) is merged per ray by t (ties: list a
 * first), as for a ray shared by the human and the object field.  t_stop > 0
 * drops samples with T_i < t_stop (render only).
 * ---------------------------------------------------------------------- */
typedef struct {                 /* one ray-major sample list */
    const int32_t *off;          /* [n_rays+1] */
    const float *sigma;          /* [n] */
    const float *rgb;            /* [n][3] */
    const float *t;              /* [n] */
    const float *dt;             /* [n] */
} nvr_samples;

nvr_status nvr_composite_fwd(int64_t n_rays, const nvr_samples *a, const nvr_samples *b,
                             float t_stop, float *C, float *D, float *TN,
                             nvr_stream stream);

/* Closed-form backward: dsigma_i = dt_i (T_{i+1} u_i - sum_{k>i} w_k u_k),
 * drgb_i = w_i dC, u_i = c_i.dC + t_i dD.  Outputs per list (overwritten);
 * b outputs nullable iff b is. */
nvr_status nvr_composite_bwd(int64_t n_rays, const nvr_samples *a, const nvr_samples *b,
                             const float *C, const float *D, const float *dC,
                             const float *dD, float *dsigma_a, float *drgb_a,
                             float *dsigma_b, float *drgb_b, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Loss (Sec. 4.3, Eq. 8, read as squared L2 on colour and depth, mean over
 * rays): L = (1/R) sum_r M_r (|C-C*|^2 + lambda_d (D-D*)^2).  Writes
 * loss_dev[0] (overwritten), dC, dD (overwritten) times loss_scale_dev[0]
 * (nullable = 1).  D_t and mask nullable.
 * ---------------------------------------------------------------------- */
nvr_status nvr_loss(int64_t n_rays, const float *C, const float *D, const float *C_t,
                    const float *D_t, const float *mask, float lambda_d,
                    const float *loss_scale_dev, float *loss_dev, float *dC, float *dD,
                    nvr_stream stream);

/* ------------------------------------------------------------------------
 * Adam with loss scaling (optimiser not stated in the paper; Instant-NGP's):
 * g = grad / S; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr_k (m / (1-b1^k)) / (sqrt(v / (1-b2^k)) + eps), k = state->step + 1,
 * lr_k = lr * lr_decay^(k-1).
 * skip_zero leaves entries with grad == 0 untouched.  The grad buffer is
 * zeroed after use.  If state->finite == 0 nothing but the zeroing happens.
 * copy (nullable) receives float16 / bfloat16 of the updated parameter.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t step;                /* completed updates */
    int32_t finite;              /* 1 if every gradient of this step is finite */
    float loss_scale;            /* S */
    float pad;
} nvr_train_state;               /* lives in DEVICE memory */

/* lr_decay: the learning rate of update k (1-based, k = state->step + 1) is
 * lr * lr_decay^(k-1) (an exponential schedule, as Instant-NGP decays its
 * rate); 0 or 1 keeps it constant. */
typedef struct { float lr, beta1, beta2, eps, lr_decay; } nvr_adam_desc;

/* state->finite = 1 (call before nvr_check_finite for a new step). */
nvr_status nvr_state_begin(nvr_train_state *state_dev, nvr_stream stream);
/* state->finite = 0 if any of g[n] is not finite. */
nvr_status nvr_check_finite(int64_t n, const float *g, nvr_train_state *state_dev,
                            nvr_stream stream);
nvr_status nvr_adam(const nvr_adam_desc *a, int64_t n, float *param, float *m, float *v,
                    float *grad, int32_t skip_zero, const nvr_train_state *state_dev,
                    void *copy, nvr_dtype copy_dtype, nvr_stream stream);
/* After every nvr_adam of a step: step += 1 if finite, else loss_scale /= 2. */
nvr_status nvr_state_end(nvr_train_state *state_dev, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Whole step (Sec. 4.2 / 4.3: per training iteration sample rays, warp human
 * samples, encode, run the networks, volume-render, back-propagate Eq. 8,
 * update).  One or two fields (human with warp, object) over ray ranges;
 * rays in both ranges are composited over the t-merged samples of both.
 * Precision NVR_F32: plain float32 kernels, float32 tables and parameters.
 * Precision NVR_BF16: float16 table copies + float32 masters, bf16 MFMA
 * networks, level-split encoder; transmittance, losses and gradients float32.
 * The context owns the per-sample workspace (sized on first use, grown on
 * demand) and, if graphs are on, one captured HIP graph per field set.
 * ---------------------------------------------------------------------- */
typedef struct nvr_ctx nvr_ctx;

/* Residual deformation network of a warped field in the step (Sec. 4.2,
 * hybrid deformation): the warped sample x_t moves to
 * x_c = x_t + MLP([enc_d(x_t), theta]) before the field's encoding, with the
 * network of nvr_deform_fwd (its own 16-level grid, 104 -> 4 x 128 -> 3).
 * NVR_F32 steps run its float32 kernels on the fp32 table, NVR_BF16 steps its
 * matrix-core kernels on the fp16 table copy (as the field's own encoding);
 * the backward chains the field encoding's position gradient through it into
 * the warp.  Its table and parameters are trained with the field (same Adam,
 * tables skip zero-gradient entries); the pose's gradient is left scaled by
 * the loss scale, like the node and bone gradients.  Host struct, device
 * arrays. */
typedef struct {
    nvr_grid_desc grid;          /* its encoding: levels x features = 32 */
    const float *theta;          /* [72] pose of the batch's frame */
    float *table;                /* [n_entries][2] fp32 */
    void *table_half;            /* [n_entries][2] float16 copy, 16-byte aligned (NVR_BF16;
                                    the step's Adam keeps it current) */
    float *params;               /* nvr_deform_param_count() fp32 */
    float *table_grad, *params_grad;          /* zero on entry, zeroed by the step */
    float *table_m, *table_v, *params_m, *params_v;
    float *theta_grad;           /* (acc, nullable) [72] */
} nvr_deform_state;

typedef struct {
    nvr_grid_desc grid;
    nvr_mlp_desc mlp;
    nvr_march_desc march;
    int32_t has_warp;
    nvr_warp_desc warp;
    nvr_warp_rig rig;            /* device pointers, used iff has_warp */
    int64_t ray_begin, ray_end;  /* rays this field covers */
    const uint32_t *occ;         /* occupancy bitfield (nullable iff occ_res == 0) */
    /* parameters, device: masters float32; copies used by NVR_BF16 */
    float *table;                /* [n_entries][2] */
    void *table_half;            /* [n_entries][2] float16 (NVR_BF16) */
    float *params;               /* flat */
    void *params_bf16;           /* flat bfloat16 (NVR_BF16) */
    float *table_grad, *params_grad;          /* zero on entry, zeroed by the step */
    float *table_m, *table_v, *params_m, *params_v;
    float *node_dq_grad;         /* (acc, nullable) [n_frames][n_nodes][8] */
    float *bones_grad;           /* (acc, nullable) [n_frames][n_joints][12] */
    const nvr_deform_state *deform;  /* nullable; only with has_warp */
} nvr_field;

typedef struct {
    int32_t n_fields;            /* 1 or 2 */
    nvr_dtype precision;         /* NVR_F32 or NVR_BF16 */
    int64_t n_rays;
    int64_t max_samples;         /* per-field sample capacity */
    float lambda_depth;
    nvr_adam_desc adam;
    int32_t apply_update;        /* 0: fwd + bwd only (gradients left in *_grad) */
} nvr_step_desc;

typedef struct {                 /* device pointers */
    const float *o, *d;          /* [n_rays][3] */
    const float *C_t;            /* [n_rays][3] */
    const float *D_t;            /* [n_rays] nullable */
    const float *mask;           /* [n_rays] nullable */
} nvr_batch;

nvr_status nvr_create(nvr_ctx **out, int32_t device, uint32_t flags);
#define NVR_USE_GRAPH 1u
/* NVR_AUTOTUNE: the first BF16 nvr_train_step at a new workspace capacity
 * times candidate launch shapes of its kernels on its own inputs and stream
 * (gather chunks per level group, emit chunk size and count, network and
 * compositing workgroups), keeps the fastest per field, and (re)captures its graph with
 * them.  Only shape-independent results are produced: the tuned step differs
 * from an untuned one only in the summation order of gradients. */
#define NVR_AUTOTUNE 2u
/* NVR_DETERMINISTIC: every sum of a training step is formed in an order fixed
 * by the inputs, so a step repeated on the same state and batch (eagerly or
 * from a captured graph) gives bit-identical losses, gradients and
 * parameters: the BF16 step's table gradients go through the deterministic
 * binned scatter (see nvr_encode_bwd_deterministic) and the autotuner is off
 * (launch shapes change summation groupings).  The node and bone gradients of
 * a warped field are still accumulated with float atomics (the optimiser does
 * not read them).  The network weight gradients and the loss are summed in a
 * fixed order with or without this flag.  The F32 step keeps its float
 * atomics on the table gradients either way. */
#define NVR_DETERMINISTIC 4u
void nvr_destroy(nvr_ctx *ctx);

/* Forward half: march, warp, encode, networks, composite, loss.  Writes
 * loss_dev[0], and (nullable) C_out[n_rays][3], D_out[n_rays]. */
nvr_status nvr_train_step_fwd(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                              const nvr_batch *b, nvr_train_state *state_dev,
                              float *loss_dev, float *C_out, float *D_out, nvr_stream stream);
/* Backward half + update, using what nvr_train_step_fwd left in the context. */
nvr_status nvr_train_step_bwd(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                              const nvr_batch *b, nvr_train_state *state_dev,
                              nvr_stream stream);
/* Both halves; with NVR_USE_GRAPH the sequence is captured once per
 * (descriptor, field, batch) set and replayed. */
nvr_status nvr_train_step(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                          const nvr_batch *b, nvr_train_state *state_dev, float *loss_dev,
                          nvr_stream stream);
/* Launch shapes in use for `field` (0 or 1): shape[0] gather chunks per level
 * group, [1] network forward workgroups, [2] network backward workgroups,
 * [3] emit chunks per level group, [4] compositing workgroups, [5] 1 if
 * tuned, [6] emit samples per chunk (256, 512 or 1024); 0 = built-in default.
 * shape is a host array of 7. */
nvr_status nvr_launch_shape(const nvr_ctx *ctx, int32_t field, int32_t *shape);

/* Total kept samples of field `field` in the last forward (synchronises
 * `stream`); count is a host pointer. */
nvr_status nvr_last_sample_count(nvr_ctx *ctx, int32_t field, int64_t *count,
                                 nvr_stream stream);

/* Forward-only render of rays o, d (device, [n_rays][3]) over every field
 * (ranges ignored: each field marches every ray; two fields are t-merged),
 * dropping samples with T_i < t_stop.  Uses each field's fp16 / bf16 copies
 * when precision is NVR_BF16.  rgb[n_rays][3], depth[n_rays]. */
nvr_status nvr_render(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                      int64_t n_rays, const float *o, const float *d, float t_stop,
                      float *rgb, float *depth, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Occupancy-grid upkeep.  The fields' back-end (Instant-NGP's, Sec. 4.3)
 * keeps the marcher's bitfield current from a decayed density grid; the paper
 * states none of its steps, and the reading is Instant-NGP's published grid at
 * one scale.  One update, all on `stream`:
 *   grid <- decay * grid (every cell; decay in [0, 1], 0.95 in that method);
 *   grid[cells[i]] <- max(grid[cells[i]], sigma(points[i])) for i < m, sigma
 *     being the field's density from the training step's encode and density
 *     network (NVR_F32: fp32 table and kernels; NVR_BF16: fp16 table copy,
 *     fp16 network forward from the fp32 masters); cells outside the grid are
 *     ignored, repeated cells take the largest density;
 *   *tau <- min(tau_max, mean(grid)) (tau_max = 0.01 * 1024 / sqrt(3) in that
 *     method), the mean formed in float64 in a fixed order;
 *   bits[c >> 5] bit (c & 31) <- grid[c] > *tau for c < res^3.
 * The grid is field->march.occ_res cubed, indexed vx + res * (vy + res * vz)
 * like the bitfield; its values must be finite and non-negative.  cells [m]
 * int32, points [m][3] float32 world positions (each inside its cell; drawn
 * by the caller), grid [res^3] float32, bits [ceil(res^3 / 32)] uint32, tau one
 * float32: all device, caller-owned.  workspace: device, 256-byte aligned, of
 * nvr_occupancy_workspace(f, precision, m) bytes.  Fields with a warp return
 * NVR_EUNSUPPORTED (their occupancy lives in the live space). */
size_t nvr_occupancy_workspace(const nvr_field *f, int32_t precision, int64_t m);
nvr_status nvr_occupancy_update(const nvr_field *f, int32_t precision, int64_t m,
                                const int32_t *cells, const float *points, float decay,
                                float tau_max, float *grid, uint32_t *bits, float *tau,
                                void *workspace, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Live look-up table of the fast neighbour search (Sec. 4.2, "On-the-fly
 * Radiance Fields").  A canonical KNN field lists the nearest graph nodes of
 * every canonical voxel; per frame, each canonical voxel centre
 * v_k = canon_min + (i + 1/2) (canon_max - canon_min) / canon_res per axis
 * (k = ix + canon_res (iy + canon_res iz)) is carried to the live space by the
 * node blend of Eq. 1, and the live voxel it lands in records k:
 *   w_j = exp(-(|v_k - x_j|^2 - d_min^2) / r_ed^2) over the listed nodes
 *     (d_min the nearest listed one: a common scale the normalised blend
 *     ignores), sign-aligned to the first listed node's rotation part,
 *   c = sum_j w_j dq_j / |real part|, v~ = R(c_r) v_k + 2 vec(c_d conj(c_r)),
 *   live voxel floor((v~ - live_min) live_res / (live_max - live_min));
 * points outside the live box are dropped, and a live voxel reached by several
 * canonical voxels keeps the largest k, one reached by none holds -1.  The
 * arithmetic is float32 (fused multiply-adds, the hardware exponential and
 * reciprocal square root; the antipodal sign is taken without fusion), so a
 * voxel whose live position lies within rounding distance of a live-voxel face
 * may land on either side; the result does not depend on the launch order.
 * knn [canon_res^3][k_nodes] uint16 node ids, nearest first (an id >= n_nodes,
 * e.g. 0xFFFF, marks "none"; a voxel whose first id is none is not carried);
 * node_canon [n_nodes][3] canonical node positions; node_dq [n_nodes][8] the
 * frame's unit node dual quaternions (w, x, y, z real part, then dual part);
 * lut [live_res^3] int32 output (overwritten): all device, caller-owned.
 * Errors: NVR_EINVAL for resolutions outside 1..1024, k_nodes outside 1..8,
 * n_nodes outside 1..65535, r_ed <= 0, an empty box, NULL or misaligned
 * arrays. */
typedef struct {
    float canon_min[3], canon_max[3];
    float live_min[3], live_max[3];
    int32_t canon_res, live_res;
    int32_t k_nodes, n_nodes;
    float r_ed;                   /* node influence radius r (0.1 in Sec. 4.1) */
} nvr_lut_desc;
nvr_status nvr_live_lut(const nvr_lut_desc *d, const uint16_t *knn, const float *node_canon,
                        const float *node_dq, int32_t *lut, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Pose-conditioned deformation network (Sec. 4.2, hybrid deformation; widths
 * in Sec. 4.3): x_can = x + MLP([enc(x), theta]) with enc a multiresolution
 * hash encoding of its own (grid `g`, 16 levels x 2 features, fp32 table) and
 * theta one 72-wide pose for all points; 104 -> 128 -> 128 -> 128
 * -> 128 -> 3, bias-free, ReLU on the hidden layers, linear output.
 * math = NVR_F32: float32 throughout (each layer one tiled product over the
 * points, weight gradients summed over point chunks in a fixed order; the
 * plain reference path).  math = NVR_F16: the hand-written matrix-core
 * kernels -- the encoding gathered from an fp16 copy of the table (formed in
 * the workspace each call), fp16 weights and activations in the forward, bf16
 * products in the backward, fp32 accumulation; the pose enters as the first
 * layer's bias W0[:, 32:] theta, weight gradients are contracted over the
 * points in fixed order.  params: nvr_deform_param_count() floats (fp32
 * masters), each layer's W[out][in] row-major in order.  x [n][3], theta [72],
 * table [n_entries][2], x_can [n][3]: device.  workspace: device, 256-byte
 * aligned, nvr_deform_workspace(g, n) bytes (about 4 KB per point, enough for
 * both paths), overwritten.
 * nvr_deform_bwd recomputes the forward and, for the gradient dx_can [n][3] of
 * the output, accumulates dparams (acc), dtable (acc, 8-byte aligned; formed
 * by the binned scatter of nvr_encode_bwd_binned, same rounding), dx (acc,
 * nullable: through the encoding -- on the F16 path from the fp16 table copy,
 * as the binned scatter forms it -- plus the identity of the residual) and
 * dtheta [72] (acc, nullable, summed over the points in a fixed order).
 * Errors: NVR_EINVAL for n outside 0..2^24, NULL arrays or workspace;
 * NVR_EUNSUPPORTED for an encoding other than 16 levels x 2 features or a
 * ladder the binned scatter does not take, math other than F32 / F16
 * (NVR_EINVAL).  Every check runs before the first launch. */
size_t nvr_deform_workspace(const nvr_grid_desc *g, int64_t n);
int64_t nvr_deform_param_count(void);
nvr_status nvr_deform_fwd(const nvr_grid_desc *g, int64_t n, const float *x, const float *theta,
                          const float *table, const float *params, nvr_dtype math, float *x_can,
                          void *workspace, nvr_stream stream);
nvr_status nvr_deform_bwd(const nvr_grid_desc *g, int64_t n, const float *x, const float *theta,
                          const float *table, const float *params, nvr_dtype math,
                          const float *dx_can, float *dparams, float *dtable, float *dx,
                          float *dtheta, void *workspace, nvr_stream stream);

/* ------------------------------------------------------------------------
 * Key-frame selection (Sec. 4.2, "Online key frame selection"; weights in
 * Sec. 4.3) and the per-pixel depth-test assembly of the two fields.
 *
 * nvr_visibility -- Eq. 5 for every node of every frame: with
 * (u', v', w') = P_f (x, 1) (P_f the frame's 3 x 4 world-to-pixel projection,
 * row-major; w' the camera depth), node i of frame f is visible when w' > 0,
 * the pixel (floor(u'/w'), floor(v'/w')) lies in the width x height map and
 * |w' - depth_f[v][u]| < eps (0.01 in Sec. 4.3).  Float32, one rounding per
 * operation, no fused multiply-add, sums in the order ((P0 x + P1 y) + P2 z)
 * + P3, correctly rounded divisions.  nodes [n_frames][n_nodes][3] world
 * positions, proj [n_frames][12], depth [n_frames][height][width] (row-major,
 * camera depth), bits [n_frames][ceil(n_nodes / 32)] uint32 output (node i at
 * word i >> 5, bit i & 31; bits past n_nodes are 0): all device,
 * caller-owned.  Errors: NVR_EINVAL for n_frames outside 0..65535, n_nodes
 * outside 0..2^24, an empty or oversized map (more than 2^28 pixels), eps < 0,
 * NULL or misaligned arrays.
 *
 * nvr_human_distance -- Eq. 6 between a query frame and n pooled frames:
 * E[j] = sum_k beta[k] (pool_theta[j][k] - q_theta[k])^2
 *        + beta_vis popcount(pool_bits[j] xor q_bits) + beta_h (pool_t[j] - q_t)^2
 * (Sec. 4.3: beta 0.1 on torso joints and 0.02 on limbs, per axis-angle
 * component; beta_vis 0.01; beta_h 0.02), float32 with the popcount exact;
 * xor_count[j] (nullable) receives the popcount.  pool_theta [n][n_pose],
 * pool_bits [n][n_words] uint32, pool_t [n] frame indices, q_theta [n_pose],
 * q_bits [n_words], beta [n_pose], E [n]: all device.  Errors: NVR_EINVAL for
 * n outside 0..2^24, n_pose outside 0..4096, n_words outside 0..2^20, NULL
 * arrays.
 *
 * nvr_object_distance -- Eq. 7: E[j] = beta_d |pool_d[j] - q_d|^2
 * + beta_o (pool_t[j] - q_t)^2 (beta_d 1, beta_o 0.02), float32; pool_d
 * [n][3] object translations, pool_t [n], q_d [3], E [n]: all device.
 *
 * nvr_pool_step -- one spatial-pool decision, host only (pool, n_pool, dist,
 * action and slot are host memory): an empty pool takes the frame
 * (NVR_POOL_FIRST); otherwise the frame enters only if dist[j] (its E to
 * pooled frame j, j < *n_pool) exceeds gamma (2.5) for every j, appended while
 * *n_pool < cap (100 in Sec. 4.3; NVR_POOL_APPEND) and otherwise replacing the
 * pooled frame with the smallest E, the lowest slot on ties
 * (NVR_POOL_REPLACE); else NVR_POOL_REJECT (slot -1).  E is a distance
 * (frames enter when it is large), so "most similar" is read as smallest E.
 *
 * nvr_pool_select -- the spatial half of the spatial-temporal pool, host
 * only: the slots of the min(m, n_pool) smallest dist (m = 10 in Sec. 4.3),
 * ascending, ties by slot, into slots[]; *n_out their number.
 *
 * nvr_depth_assemble -- the per-pixel combination of two renderings by depth:
 * a field covers a pixel when its opacity alpha = 1 - T_N is >= 1/2, its
 * surface depth being depth / alpha; the pixel takes the colour and surface
 * depth of the nearer covering field (the first on ties); with none covering,
 * the colours add (both over black) and the depth is the more opaque field's
 * depth / alpha (the first's on ties; 0 when its alpha is 0).  rgb_* [n][3],
 * depth_* [n] (un-normalised, as nvr_render writes them), alpha_* [n],
 * rgb [n][3], depth [n] outputs: all device.  Errors: NVR_EINVAL for n
 * outside 0..2^31, NULL arrays. */
enum { NVR_POOL_REJECT = 0, NVR_POOL_FIRST = 1, NVR_POOL_APPEND = 2, NVR_POOL_REPLACE = 3 };
nvr_status nvr_visibility(int32_t n_frames, int32_t n_nodes, const float *nodes,
                          const float *proj, const float *depth, int32_t height, int32_t width,
                          float eps, uint32_t *bits, nvr_stream stream);
nvr_status nvr_human_distance(int32_t n, int32_t n_pose, int32_t n_words,
                              const float *pool_theta, const uint32_t *pool_bits,
                              const int32_t *pool_t, const float *q_theta, const uint32_t *q_bits,
                              int32_t q_t, const float *beta, float beta_vis, float beta_h,
                              float *E, int32_t *xor_count, nvr_stream stream);
nvr_status nvr_object_distance(int32_t n, const float *pool_d, const int32_t *pool_t,
                               const float *q_d, int32_t q_t, float beta_d, float beta_o,
                               float *E, nvr_stream stream);
nvr_status nvr_pool_step(int32_t *pool, int32_t *n_pool, int32_t cap, const float *dist,
                         int32_t frame, float gamma, int32_t *action, int32_t *slot);
nvr_status nvr_pool_select(int32_t n_pool, const float *dist, int32_t m, int32_t *slots,
                           int32_t *n_out);
nvr_status nvr_depth_assemble(int64_t n, const float *rgb_a, const float *depth_a,
                              const float *alpha_a, const float *rgb_b, const float *depth_b,
                              const float *alpha_b, float *rgb, float *depth,
                              nvr_stream stream);

/* ------------------------------------------------------------------------
 * Measurement probe (not part of the method): the random-gather ceiling the
 * hash-grid gather of Sec. 4.3's back-end is measured against.  The table
 * (device, 16-byte aligned, `bytes` long) is split into eight equal slices;
 * workgroup b serves slice b % 8 (one per XCD, as the level-split gather
 * serves level groups).  For each of the n items of each slice, `loads`
 * (a positive multiple of 4, <= 1024) independent 16-byte loads at uniformly
 * random aligned offsets of the slice are issued, and the xor of the loaded
 * words is stored to out[slice][n] (device, caller-owned, 8 n words).
 * Errors: NVR_EINVAL for n outside [0, 2^31), bad `loads`, a table under
 * 128 bytes or over 2^39 bytes, NULL or misaligned arrays. */
nvr_status nvr_probe_gather(const void *table, size_t bytes, int64_t n, int32_t loads,
                            uint32_t seed, uint32_t *out, nvr_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* NVR_H */
