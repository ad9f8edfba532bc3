// Whole training step, forward-only render and the public network entry
// points.  The context owns per-field sample workspaces (fixed capacity, so
// every launch is sized without reading the device-side sample count) and,
// with NVR_USE_GRAPH, one captured HIP graph per (descriptor, fields, batch).
#include "deform_dev.hpp"
#include "launch.hpp"
#include "scatter_dev.hpp"

#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace nvr {

struct FieldWs {
    int64_t cap = 0, n_rays = 0;
    int precision = -1;
    int has_warp = 0, n_in = 0, has_deform = 0;
    size_t mlp_bytes = 0, scatter_bytes = 0, deform_bytes = 0, jac_bytes = 0;
    void *block = nullptr;          // one allocation, carved below
    int32_t *off, *ray_id, *n_dev, *march_ws;
    float *t, *dt, *x, *xc;
    void *feat;                     // bf16 planar [8][cap][4] | f32 [cap][n_in]
    float *sigma, *rgb, *dsigma, *drgb;
    float *dfeat;                   // f32 planar [8][cap][4] | f32 [cap][n_in]
    float *dx;                      // [8][cap][3] (split) | [cap][3] (plain)
    uint32_t *jac;                  // bf16 training of a warped field: the gather's spatial
                                    // derivatives [8][cap][3 lpg] (fp16 pairs)
    void *mlp_ws;
    void *scatter_ws;               // binned table-gradient scatter (bf16 training)
    float *sh;                      // bf16 path: per-ray SH coefficients [n_rays][16]
    // deformation network (warped fields with one): deformed positions, the
    // summed gradient w.r.t. them, the gradient w.r.t. the warped positions
    float *xd, *dxd, *dxt;
    void *deform_ws;
    // launch shapes of the BF16 step's kernels (0: built-in default), set by
    // the autotuner for this capacity
    int enc_chunks = 0, mlp_fwd_blocks = 0, mlp_bwd_blocks = 0, emit_chunks = 0, emit_block = 0;
    bool tuned = false;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

}  // namespace nvr

struct nvr_ctx {
    int device = 0;
    uint32_t flags = 0;
    hipStream_t capture = nullptr;
    // second stream (default priority) on which a warped field's table-gradient
    // accumulation overlaps its chain through the deformation network and warp
    hipStream_t side = nullptr;
    hipEvent_t ev_fork[3] = {nullptr, nullptr, nullptr}, ev_join = nullptr;
    nvr::FieldWs ws[2];
    int comp_blocks = 0;           // compositing workgroups (autotuned; 0: default)
    float *ray_buf = nullptr;      // render: C, D per ray chunk
    float *loss_part = nullptr;    // one loss partial per compositing workgroup
    int64_t ray_buf_n = 0;
    std::map<std::string, nvr::GraphEntry> graphs;
};

namespace nvr {

static size_t up(size_t v) { return (v + 255) & ~size_t(255); }

static nvr_status field_check(const nvr_field *f, const nvr_step_desc *s, Net *net) {
    NVR_REQUIRE(f != nullptr, NVR_EINVAL, "field is NULL");
    NVR_TRY(check_grid(&f->grid));
    NVR_TRY(build_net(&f->mlp, net));
    NVR_REQUIRE(net->n_in == f->grid.n_levels * f->grid.n_features, NVR_EINVAL,
                "network input width %d != encoding width %d", net->n_in,
                f->grid.n_levels * f->grid.n_features);
    NVR_TRY(march_desc_check(&f->march));
    NVR_REQUIRE(f->march.occ_res == 0 || f->occ, NVR_EINVAL, "occupancy bitfield is NULL");
    NVR_REQUIRE(f->ray_begin >= 0 && f->ray_begin <= f->ray_end && f->ray_end <= s->n_rays,
                NVR_EINVAL, "field ray range outside [0, n_rays)");
    NVR_REQUIRE(f->table && f->params, NVR_EINVAL, "NULL parameter masters");
    if (s->precision == NVR_BF16) {
        NVR_REQUIRE(f->table_half && f->params_bf16, NVR_EINVAL, "NULL fp16 / bf16 copies");
        NVR_REQUIRE(f->grid.n_levels == 16, NVR_EUNSUPPORTED,
                    "the bf16 step uses the planar 16-level layout");
        NVR_TRY(mfma_check(*net));
    }
    if (f->has_warp) {
        NVR_REQUIRE(f->warp.n_frames >= 1, NVR_EINVAL, "warp n_frames < 1");
    }
    if (f->deform) {
        const nvr_deform_state *D = f->deform;
        NVR_REQUIRE(f->has_warp, NVR_EINVAL, "a deformation network needs the warp");
        NVR_TRY(deform_check(&D->grid, s->max_samples));
        NVR_REQUIRE(D->theta && D->table && D->params, NVR_EINVAL,
                    "NULL deformation pose, table or parameters");
        NVR_REQUIRE(s->precision != NVR_BF16 || (D->table_half && aligned(D->table_half, 16)),
                    NVR_EINVAL, "NULL or misaligned fp16 deformation table copy");
        NVR_REQUIRE(aligned(D->table, 8) && aligned(D->theta, 4) && aligned(D->params, 4),
                    NVR_EINVAL, "misaligned deformation arrays");
    }
    return NVR_OK;
}

// positions the field's encoding reads: deformed, warped or marched
static const float *enc_pos(const nvr_field *f, const FieldWs &w) {
    return f->deform ? w.xd : f->has_warp ? w.xc : w.x;
}

static bool deterministic(const nvr_ctx *ctx) { return (ctx->flags & NVR_DETERMINISTIC) != 0; }

static nvr_status ensure_ws(nvr_ctx *ctx, int k, const nvr_field *f, const Net &net, int precision,
                            int64_t n_rays, int64_t cap, bool train) {
    FieldWs &w = ctx->ws[k];
    const size_t mlp_bytes = precision == NVR_BF16 ? mfma_ws_bytes(net, cap) : plain_workspace(net, cap);
    const GridParams gp = make_grid_params(&f->grid);
    const size_t scatter_bytes =
        (train && precision == NVR_BF16)
            ? (deterministic(ctx) ? scatter_det_ws_bytes(gp, cap) : scatter_ws_bytes(gp, cap))
            : 0;
    const size_t jac_bytes =
        (train && precision == NVR_BF16 && f->has_warp)
            ? sizeof(uint32_t) * 3 * kXcds * (size_t)((f->grid.n_levels + kXcds - 1) / kXcds) * cap
            : 0;
    const int has_deform = f->deform ? 1 : 0;
    if (has_deform) NVR_TRY(deform_setup());
    const size_t deform_bytes =
        has_deform ? deform_ws_bytes(&f->deform->grid, cap, precision == NVR_BF16,
                                     deterministic(ctx))
                   : 0;
    if (w.block && w.cap >= cap && w.n_rays >= n_rays && w.precision == precision &&
        w.has_warp == f->has_warp && w.n_in == net.n_in && w.mlp_bytes >= mlp_bytes &&
        w.scatter_bytes >= scatter_bytes && w.has_deform == has_deform &&
        w.deform_bytes >= deform_bytes && w.jac_bytes >= jac_bytes)
        return NVR_OK;
    if (w.block) {
        NVR_HIP(hipDeviceSynchronize());
        NVR_HIP(hipFree(w.block));
        w.block = nullptr;
        // graphs reference the old buffers
        for (auto &g : ctx->graphs) {
            if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
            if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
        }
        ctx->graphs.clear();
    }
    const bool bf = precision == NVR_BF16;
    const int nin = net.n_in;
    size_t sz[23] = {
        sizeof(int32_t) * (size_t)(n_rays + 1),             // off
        sizeof(int32_t) * (size_t)cap,                      // ray_id
        sizeof(int32_t) * 4,                                // n_dev
        march_ws_bytes(n_rays),                             // march scratch
        sizeof(float) * (size_t)cap,                        // t
        sizeof(float) * (size_t)cap,                        // dt
        sizeof(float) * 3 * (size_t)cap,                    // x
        f->has_warp ? sizeof(float) * 3 * (size_t)cap : 0,  // xc
        bf ? sizeof(uint16_t) * 32 * (size_t)cap : sizeof(float) * nin * (size_t)cap,  // feat
        sizeof(float) * (size_t)cap,                        // sigma
        sizeof(float) * 3 * (size_t)cap,                    // rgb
        sizeof(float) * (size_t)cap,                        // dsigma
        sizeof(float) * 3 * (size_t)cap,                    // drgb
        sizeof(float) * (bf ? 32 : nin) * (size_t)cap,      // dfeat
        f->has_warp ? sizeof(float) * 3 * (bf ? kXcds : 1) * (size_t)cap : 0,  // dx
        mlp_bytes,                                                             // mlp
        scatter_bytes,                                                         // scatter
        bf ? sizeof(float) * 16 * (size_t)n_rays : 0,                          // sh
        has_deform ? sizeof(float) * 3 * (size_t)cap : 0,                      // xd
        has_deform ? sizeof(float) * 3 * (size_t)cap : 0,                      // dxd
        has_deform ? sizeof(float) * 3 * (size_t)cap : 0,                      // dxt
        deform_bytes,                                                          // deform
        jac_bytes,                                                             // jac
    };
    size_t total = 0;
    for (size_t s : sz) total += up(s);
    void *blk = nullptr;
    hipError_t e = hipMalloc(&blk, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation of %zu bytes failed: %s", total, hipGetErrorString(e));
        return NVR_ENOMEM;
    }
    char *p = (char *)blk;
    void *ptr[23];
    for (int i = 0; i < 23; ++i) {
        ptr[i] = sz[i] ? p : nullptr;
        p += up(sz[i]);
    }
    w.block = blk;
    w.cap = cap;
    w.n_rays = n_rays;
    w.precision = precision;
    w.has_warp = f->has_warp;
    w.n_in = net.n_in;
    w.mlp_bytes = mlp_bytes;
    w.scatter_bytes = scatter_bytes;
    w.has_deform = has_deform;
    w.deform_bytes = deform_bytes;
    w.jac_bytes = jac_bytes;
    w.off = (int32_t *)ptr[0];
    w.ray_id = (int32_t *)ptr[1];
    w.n_dev = (int32_t *)ptr[2];
    w.march_ws = (int32_t *)ptr[3];
    w.t = (float *)ptr[4];
    w.dt = (float *)ptr[5];
    w.x = (float *)ptr[6];
    w.xc = (float *)ptr[7];
    w.feat = ptr[8];
    w.sigma = (float *)ptr[9];
    w.rgb = (float *)ptr[10];
    w.dsigma = (float *)ptr[11];
    w.drgb = (float *)ptr[12];
    w.dfeat = (float *)ptr[13];
    w.dx = (float *)ptr[14];
    w.mlp_ws = ptr[15];
    w.scatter_ws = ptr[16];
    w.sh = (float *)ptr[17];
    w.xd = (float *)ptr[18];
    w.dxd = (float *)ptr[19];
    w.dxt = (float *)ptr[20];
    w.deform_ws = ptr[21];
    w.jac = (uint32_t *)ptr[22];
    w.enc_chunks = w.mlp_fwd_blocks = w.mlp_bwd_blocks = w.emit_chunks = w.emit_block = 0;
    w.tuned = false;
    return NVR_OK;
}

// march -> [warp] -> encode -> networks for one field over rays [begin, end)
static nvr_status field_forward(nvr_ctx *ctx, int k, const nvr_field *f, const Net &net,
                                int precision, int64_t n_rays, int64_t begin, int64_t end,
                                const float *o, const float *d, bool train, hipStream_t st) {
    FieldWs &w = ctx->ws[k];
    const int64_t cap = w.cap;
    NVR_TRY(run_march(&f->march, n_rays, begin, end, o, d, f->occ, cap, w.off, w.ray_id, w.t, w.dt,
                      w.x, w.n_dev, w.march_ws, st));
    const float *pos = w.x;
    if (f->has_warp) {
        NVR_TRY(run_warp_fwd(&f->warp, &f->rig, cap, w.n_dev, w.x, w.xc, st));
        pos = w.xc;
    }
    if (f->deform) {
        const nvr_deform_state *D = f->deform;
        NVR_TRY(deform_fwd_dev(&D->grid, precision == NVR_BF16, w.n_dev, cap, w.xc, D->theta,
                               D->table, D->table_half, D->params, w.xd, train,
                               deterministic(ctx), w.deform_ws, st));
        pos = w.xd;
    }
    const GridParams gp = make_grid_params(&f->grid);
    if (precision == NVR_BF16) {
        // a training forward also counts the table-gradient scatter's tiles
        // (the deterministic scatter forms its own counts per chunk)
        TileCounter counter{};
        const bool count = train && w.scatter_ws != nullptr && !deterministic(ctx);
        if (count) {
            counter = scatter_counter(gp, w.scatter_ws);
            NVR_TRY(launch_counter_reset(gp, w.scatter_ws, st));
        }
        // fp16 features and fp16 forward; the networks' backward products run in bf16
        // (and, for a warped field, stores the spatial derivatives its position
        // gradient needs)
        NVR_TRY(launch_encode_fwd(gp, 0, w.n_dev, cap, pos, f->table_half, NVR_F16, w.feat, NVR_F16,
                                  true, st, count ? &counter : nullptr, w.enc_chunks,
                                  train && f->has_warp ? w.jac : nullptr));
        // the colour network's direction encoding, once per ray
        NVR_TRY(launch_sh_rays(net, n_rays, d, w.sh, st));
        NVR_TRY(mfma_fwd(net, 0, w.n_dev, cap, (const uint16_t *)w.feat, true, d, w.ray_id,
                         f->params, true, w.sigma, w.rgb, st, w.mlp_fwd_blocks, w.sh));
    } else {
        NVR_TRY(launch_encode_fwd(gp, 0, w.n_dev, cap, pos, f->table, NVR_F32, w.feat, NVR_F32, false,
                                  st));
        PlainView F{(float *)w.feat, 1, net.n_in};
        NVR_TRY(plain_fwd(net, 0, w.n_dev, cap, F, d, w.ray_id, f->params, w.sigma, w.rgb,
                          (float *)w.mlp_ws, st));
    }
    return NVR_OK;
}

static nvr_samples samples_of(const FieldWs &w) {
    return nvr_samples{w.off, w.sigma, w.rgb, w.t, w.dt};
}

static nvr_status step_check(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                             const nvr_batch *b, Net *nets) {
    NVR_REQUIRE(ctx && s && fields && b, NVR_EINVAL, "NULL argument");
    NVR_REQUIRE(s->n_fields == 1 || s->n_fields == 2, NVR_EINVAL, "n_fields must be 1 or 2");
    NVR_REQUIRE(s->precision == NVR_F32 || s->precision == NVR_BF16, NVR_EINVAL,
                "precision must be F32 or BF16");
    NVR_REQUIRE(s->n_rays >= 1 && s->n_rays < (1ll << 31), NVR_EINVAL, "n_rays out of range");
    NVR_REQUIRE(s->max_samples >= 1 && s->max_samples < (1ll << 31), NVR_EINVAL,
                "max_samples out of range");
    NVR_REQUIRE(b->o && b->d && b->C_t, NVR_EINVAL, "NULL batch array");
    const nvr_adam_desc &a = s->adam;
    NVR_REQUIRE(a.lr > 0.f && a.beta1 >= 0.f && a.beta1 < 1.f && a.beta2 >= 0.f &&
                    a.beta2 < 1.f && a.eps >= 0.f && a.lr_decay >= 0.f && a.lr_decay <= 1.f,
                NVR_EINVAL, "bad Adam hyper-parameters");
    for (int k = 0; k < s->n_fields; ++k) NVR_TRY(field_check(fields[k], s, &nets[k]));
    return NVR_OK;
}

static nvr_status enqueue_fwd(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                              const nvr_batch *b, const Net *nets, nvr_train_state *state,
                              float *loss, float *C_out, float *D_out, hipStream_t st) {
    for (int k = 0; k < s->n_fields; ++k)
        NVR_TRY(field_forward(ctx, k, fields[k], nets[k], s->precision, s->n_rays, fields[k]->ray_begin,
                              fields[k]->ray_end, b->o, b->d, /*train=*/true, st));
    const nvr_samples a = samples_of(ctx->ws[0]);
    nvr_samples bb;
    if (s->n_fields == 2) bb = samples_of(ctx->ws[1]);
    return launch_composite_loss(s->n_rays, a, s->n_fields == 2 ? &bb : nullptr, b->C_t, b->D_t, b->mask,
                                 s->lambda_depth, state, loss, C_out, D_out, ctx->ws[0].dsigma,
                                 ctx->ws[0].drgb, s->n_fields == 2 ? ctx->ws[1].dsigma : nullptr,
                                 s->n_fields == 2 ? ctx->ws[1].drgb : nullptr, st, ctx->comp_blocks,
                                 ctx->loss_part);
}

// Position gradient of the encoding (n_parts partial arrays in w.dx) back
// through the deformation network, if any, and the warp.
static nvr_status warp_chain_bwd(nvr_ctx *ctx, const nvr_field *f, FieldWs &w, int n_parts,
                                 hipStream_t st, const ScatterTail *tail = nullptr) {
    const int64_t cap = w.cap;
    if (!f->deform)
        return run_warp_bwd(&f->warp, &f->rig, cap, w.n_dev, w.x, w.dx, n_parts, 3 * cap,
                            f->node_dq_grad, f->bones_grad, st);
    const nvr_deform_state *D = f->deform;
    const float *dxd = w.dx;
    if (n_parts > 1) {
        NVR_TRY(launch_sum_parts(w.n_dev, cap, n_parts, 3 * cap, w.dx, w.dxd, st));
        dxd = w.dxd;
    }
    NVR_TRY(launch_fill_zero(w.dxt, 3 * cap, st));
    NVR_TRY(deform_bwd_dev(&D->grid, w.precision == NVR_BF16, w.n_dev, cap, w.xc, D->theta,
                           D->table, D->table_half, D->params, dxd, D->params_grad,
                           D->table_grad, w.dxt, D->theta_grad, deterministic(ctx), w.deform_ws,
                           st, tail));
    return run_warp_bwd(&f->warp, &f->rig, cap, w.n_dev, w.x, w.dxt, 1, 3 * cap, f->node_dq_grad,
                        f->bones_grad, st);
}

// A warped BF16 field's table-gradient accumulation (and its deformation
// network's) runs on the context's second stream, overlapping the chain
// through the network and the warp, which only needs the emit pass's position
// gradient; the deterministic mode keeps one stream.
static bool overlap(const nvr_ctx *ctx, const nvr_field *f) {
    return f->has_warp && ctx->side != nullptr && !deterministic(ctx);
}

static nvr_status enqueue_bwd(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                              const nvr_batch *b, const Net *nets, nvr_train_state *state,
                              hipStream_t st) {
    const ScatterTail tails[2] = {{ctx->side, ctx->ev_fork[0]}, {ctx->side, ctx->ev_fork[1]}};
    bool forked = false;
    // beside a warped field, a field without a warp runs its whole backward on
    // the second stream (it is independent of the warped field's), first
    bool any_warp = false;
    for (int k = 0; k < s->n_fields; ++k) any_warp |= overlap(ctx, fields[k]);
    const bool side_plain = any_warp && s->n_fields > 1 && s->precision == NVR_BF16;
    if (side_plain) {
        NVR_HIP(hipEventRecord(ctx->ev_fork[2], st));
        NVR_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork[2], 0));
        forked = true;
    }
    int order[2] = {0, 1};
    if (side_plain && fields[0]->has_warp) order[0] = 1, order[1] = 0;
    for (int i = 0; i < s->n_fields; ++i) {
        const int k = s->n_fields > 1 ? order[i] : i;
        const nvr_field *f = fields[k];
        FieldWs &w = ctx->ws[k];
        const int64_t cap = w.cap;
        const float *pos = enc_pos(f, w);
        const GridParams gp = make_grid_params(&f->grid);
        if (s->precision == NVR_BF16) {
            const hipStream_t fs = side_plain && !f->has_warp ? ctx->side : st;
            NVR_TRY(mfma_bwd(nets[k], 0, w.n_dev, cap, (const uint16_t *)w.feat, true, b->d, w.ray_id,
                             f->params, true, w.dsigma, w.drgb, f->params_grad, w.dfeat, w.mlp_ws,
                             fs, w.mlp_bwd_blocks, w.sh));
            if (deterministic(ctx))
                NVR_TRY(launch_scatter_det(gp, 0, w.n_dev, cap, pos, f->table_half, w.dfeat,
                                           f->table_grad, f->has_warp ? w.dx : nullptr,
                                           w.scatter_ws, st, f->has_warp ? w.jac : nullptr));
            else
                NVR_TRY(launch_scatter(gp, 0, w.n_dev, cap, pos, f->table_half, w.dfeat,
                                       f->table_grad, f->has_warp ? w.dx : nullptr, w.scatter_ws,
                                       fs, /*counted=*/true, w.emit_chunks, w.emit_block,
                                       f->has_warp ? w.jac : nullptr,
                                       overlap(ctx, f) ? &tails[0] : nullptr));
            if (f->has_warp)
                NVR_TRY(warp_chain_bwd(ctx, f, w, kXcds, st, overlap(ctx, f) ? &tails[1] : nullptr));
            forked |= overlap(ctx, f);
        } else {
            PlainView F{(float *)w.feat, 1, nets[k].n_in};
            PlainView dF{w.dfeat, 1, nets[k].n_in};
            NVR_TRY(plain_bwd(nets[k], 0, w.n_dev, cap, F, f->params, w.sigma, w.rgb, w.dsigma, w.drgb,
                              f->params_grad, dF, true, (float *)w.mlp_ws, st));
            if (f->has_warp) NVR_TRY(launch_fill_zero(w.dx, 3 * cap, st));
            NVR_TRY(launch_encode_bwd(gp, 0, w.n_dev, cap, pos, f->table, NVR_F32, w.dfeat,
                                      f->table_grad, f->has_warp ? w.dx : nullptr, false, st));
            if (f->has_warp) NVR_TRY(warp_chain_bwd(ctx, f, w, 1, st));
        }
    }
    if (forked) {   // the second stream's work joins the caller's stream here
        NVR_HIP(hipEventRecord(ctx->ev_join, ctx->side));
        NVR_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
    }
    if (!s->apply_update) return NVR_OK;
    NVR_TRY(launch_state_begin(state, st));
    for (int k = 0; k < s->n_fields; ++k) {
        const nvr_field *f = fields[k];
        NVR_TRY(launch_check_finite(f->grid.offset[f->grid.n_levels] * 2, f->table_grad, state, st));
        NVR_TRY(launch_check_finite(nets[k].woff[nets[k].n_layers], f->params_grad, state, st));
        if (const nvr_deform_state *D = f->deform) {
            NVR_TRY(launch_check_finite(D->grid.offset[D->grid.n_levels] * 2, D->table_grad,
                                        state, st));
            NVR_TRY(launch_check_finite(deform_param_count(), D->params_grad, state, st));
        }
    }
    const AdamParams ap = adam_params(s->adam);
    const bool bf = s->precision == NVR_BF16;
    for (int k = 0; k < s->n_fields; ++k) {
        const nvr_field *f = fields[k];
        NVR_TRY(launch_adam(ap, f->grid.offset[f->grid.n_levels] * 2, f->table, f->table_m, f->table_v,
                            f->table_grad, 1, state, bf ? f->table_half : nullptr, NVR_F16, st));
        NVR_TRY(launch_adam(ap, nets[k].woff[nets[k].n_layers], f->params, f->params_m, f->params_v,
                            f->params_grad, 0, state, bf ? f->params_bf16 : nullptr, NVR_BF16, st));
        if (const nvr_deform_state *D = f->deform) {
            NVR_TRY(launch_adam(ap, D->grid.offset[D->grid.n_levels] * 2, D->table, D->table_m,
                                D->table_v, D->table_grad, 1, state,
                                bf ? D->table_half : nullptr, NVR_F16, st));
            NVR_TRY(launch_adam(ap, deform_param_count(), D->params, D->params_m, D->params_v,
                                D->params_grad, 0, state, nullptr, NVR_BF16, st));
        }
    }
    return launch_state_end(state, st);
}

static nvr_status prepare(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                          const Net *nets) {
    NVR_HIP(hipSetDevice(ctx->device));
    if (s->precision == NVR_BF16)
        for (int k = 0; k < s->n_fields; ++k) {
            NVR_TRY(scatter_check(make_grid_params(&fields[k]->grid)));
            NVR_REQUIRE((size_t)s->max_samples * fields[k]->grid.n_levels * 8 < (1ull << 32),
                        NVR_EINVAL, "max_samples too large for the binned scatter");
        }
    for (int k = 0; k < s->n_fields; ++k)
        NVR_TRY(ensure_ws(ctx, k, fields[k], nets[k], s->precision, s->n_rays, s->max_samples, true));
    if (s->precision == NVR_BF16)
        for (int k = 0; k < s->n_fields; ++k)
            NVR_REQUIRE(fields[k]->params_m && fields[k]->params_v && fields[k]->table_m &&
                            fields[k]->table_v && fields[k]->table_grad && fields[k]->params_grad,
                        NVR_EINVAL, "NULL optimiser buffers");
    for (int k = 0; k < s->n_fields; ++k)
        if (const nvr_deform_state *D = fields[k]->deform) {
            NVR_REQUIRE(D->table_grad && D->params_grad && aligned(D->table_grad, 8), NVR_EINVAL,
                        "NULL or misaligned deformation gradients");
            NVR_REQUIRE(!s->apply_update ||
                            (D->table_m && D->table_v && D->params_m && D->params_v),
                        NVR_EINVAL, "NULL deformation optimiser buffers");
        }
    return NVR_OK;
}

// ---------------------------------------------------------------- autotuner
// Best of `reps` timed launches (after one untimed) on stream st.
template <class F>
static nvr_status time_best(hipStream_t st, F &&launch, float *best_ms, int reps = 5) {
    hipEvent_t e0, e1;
    NVR_HIP(hipEventCreate(&e0));
    NVR_HIP(hipEventCreate(&e1));
    nvr_status r = launch();
    float best = 1e30f;
    for (int i = 0; i < reps && r == NVR_OK; ++i) {
        (void)hipEventRecord(e0, st);
        r = launch();
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = ms < best ? ms : best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_ms = best;
    return r;
}

// Picks the candidate of `cands` (n of them) with the shortest launch; a later
// candidate must beat the one held by more than 1% (timing noise between
// near-equal shapes would otherwise decide).
template <class F>
static nvr_status pick(hipStream_t st, const int *cands, int n, int *out, F &&launch_with) {
    float best = 1e30f;
    int arg = cands[0];
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        NVR_TRY(time_best(st, [&] { return launch_with(cands[i]); }, &ms));
        if (ms < 0.99f * best) {
            best = ms;
            arg = cands[i];
        }
    }
    *out = arg;
    return NVR_OK;
}

// Tunes the launch shapes of the BF16 step on its real inputs (eager, before
// any graph capture): one forward fills the sample buffers, then every
// tunable kernel is timed per candidate shape.  Only launches without side
// effects on the optimiser state are repeated: the gather (its tile counts
// are reset each time), the network forward, the compositing + loss (it
// zeroes the loss first), the network backward without the reduction into
// the weight gradients, and the scatter's scan + emit.  Results do not
// depend on the shapes except for the summation order of the gradients.
static nvr_status autotune(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                           const nvr_batch *b, const Net *nets, nvr_train_state *state,
                           float *loss, hipStream_t st) {
    NVR_TRY(enqueue_fwd(ctx, s, fields, b, nets, state, loss, nullptr, nullptr, st));
    // candidates in order of preference: the first is kept unless another is
    // more than 1% faster (the first ones are best inside the whole step at
    // millions of samples)
    static const int enc[] = {2048, 1024, 512, 256};
    static const int mlp_f[] = {2048, 1024, 512, 256};
    static const int mlp_b[] = {512, 256, 128};
    // emit: samples per chunk * kShape + chunks per level group
    constexpr int kShape = 100000;
    static const int emit[] = {512 * kShape + 1024, 512 * kShape + 512, 512 * kShape + 256,
                               512 * kShape + 128, 512 * kShape + 64, 1024 * kShape + 128,
                               1024 * kShape + 64, 1024 * kShape + 32, 256 * kShape + 1024,
                               256 * kShape + 2048};
    static const int comp[] = {4096, 16384, 65536};
    for (int k = 0; k < s->n_fields; ++k) {
        const nvr_field *f = fields[k];
        FieldWs &w = ctx->ws[k];
        const int64_t cap = w.cap;
        const float *pos = enc_pos(f, w);
        const GridParams gp = make_grid_params(&f->grid);
        const TileCounter counter = scatter_counter(gp, w.scatter_ws);
        NVR_TRY(pick(st, enc, 4, &w.enc_chunks, [&](int c) {
            NVR_TRY(launch_counter_reset(gp, w.scatter_ws, st));
            return launch_encode_fwd(gp, 0, w.n_dev, cap, pos, f->table_half, NVR_F16, w.feat,
                                     NVR_F16, true, st, &counter, c,
                                     f->has_warp ? w.jac : nullptr);
        }));
        NVR_TRY(pick(st, mlp_f, 4, &w.mlp_fwd_blocks, [&](int c) {
            return mfma_fwd(nets[k], 0, w.n_dev, cap, (const uint16_t *)w.feat, true, b->d,
                            w.ray_id, f->params, true, w.sigma, w.rgb, st, c, w.sh);
        }));
    }
    const nvr_samples sa = samples_of(ctx->ws[0]);
    nvr_samples sb;
    if (s->n_fields == 2) sb = samples_of(ctx->ws[1]);
    NVR_TRY(pick(st, comp, 3, &ctx->comp_blocks, [&](int c) {
        return launch_composite_loss(s->n_rays, sa, s->n_fields == 2 ? &sb : nullptr, b->C_t, b->D_t,
                                     b->mask, s->lambda_depth, state, loss, nullptr, nullptr,
                                     ctx->ws[0].dsigma, ctx->ws[0].drgb,
                                     s->n_fields == 2 ? ctx->ws[1].dsigma : nullptr,
                                     s->n_fields == 2 ? ctx->ws[1].drgb : nullptr, st, c,
                                     ctx->loss_part);
    }));
    for (int k = 0; k < s->n_fields; ++k) {
        const nvr_field *f = fields[k];
        FieldWs &w = ctx->ws[k];
        const int64_t cap = w.cap;
        const float *pos = enc_pos(f, w);
        const GridParams gp = make_grid_params(&f->grid);
        NVR_TRY(pick(st, mlp_b, 3, &w.mlp_bwd_blocks, [&](int c) {
            return mfma_bwd(nets[k], 0, w.n_dev, cap, (const uint16_t *)w.feat, true, b->d, w.ray_id,
                            f->params, true, w.dsigma, w.drgb, nullptr, w.dfeat, w.mlp_ws, st, c,
                            w.sh);
        }));
        int e = 0;
        NVR_TRY(pick(st, emit, 10, &e, [&](int c) {
            return launch_scatter_emit_only(gp, 0, w.n_dev, cap, pos, f->table_half, w.dfeat,
                                            w.scatter_ws, st, c % kShape, c / kShape);
        }));
        w.emit_chunks = e % kShape;
        w.emit_block = e / kShape;
        w.tuned = true;
    }
    return NVR_OK;
}

static std::string graph_key(const nvr_step_desc *s, nvr_field *const *fields, const nvr_batch *b,
                             const nvr_train_state *state, const float *loss) {
    std::string k;
    k.append((const char *)s, sizeof(*s));
    for (int i = 0; i < s->n_fields; ++i) {
        k.append((const char *)fields[i], sizeof(nvr_field));
        if (fields[i]->deform) k.append((const char *)fields[i]->deform, sizeof(nvr_deform_state));
    }
    k.append((const char *)b, sizeof(*b));
    k.append((const char *)&state, sizeof(state));
    k.append((const char *)&loss, sizeof(loss));
    return k;
}

}  // namespace nvr

using namespace nvr;

extern "C" nvr_status nvr_create(nvr_ctx **out, int32_t device, uint32_t flags) {
    clear_error();
    NVR_REQUIRE(out != nullptr, NVR_EINVAL, "out is NULL");
    int n = 0;
    NVR_HIP(hipGetDeviceCount(&n));
    NVR_REQUIRE(device >= 0 && device < n, NVR_EINVAL, "device %d out of range (%d devices)", device, n);
    nvr_ctx *c = new nvr_ctx();
    c->device = device;
    c->flags = flags;
    NVR_HIP(hipSetDevice(device));
    {
        hipError_t e = hipMalloc(&c->loss_part, sizeof(float) * kMaxLossBlocks);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete c;
            set_error("loss partials allocation failed: %s", hipGetErrorString(e));
            return NVR_ENOMEM;
        }
    }
    if (flags & NVR_USE_GRAPH) {
        hipError_t e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            set_error("hipStreamCreate failed: %s", hipGetErrorString(e));
            return NVR_EHIP;
        }
    }
    {
        hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        for (int i = 0; i < 3 && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&c->ev_fork[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) {
            nvr_destroy(c);
            set_error("stream / event creation failed: %s", hipGetErrorString(e));
            return NVR_EHIP;
        }
    }
    *out = c;
    return NVR_OK;
}

extern "C" void nvr_destroy(nvr_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &g : ctx->graphs) {
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
    }
    for (auto &w : ctx->ws)
        if (w.block) (void)hipFree(w.block);
    if (ctx->ray_buf) (void)hipFree(ctx->ray_buf);
    if (ctx->loss_part) (void)hipFree(ctx->loss_part);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    for (hipEvent_t e : ctx->ev_fork)
        if (e) (void)hipEventDestroy(e);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    delete ctx;
}

extern "C" nvr_status nvr_train_step_fwd(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                                         const nvr_batch *b, nvr_train_state *state_dev,
                                         float *loss_dev, float *C_out, float *D_out,
                                         nvr_stream stream) {
    clear_error();
    Net nets[2];
    NVR_TRY(step_check(ctx, s, fields, b, nets));
    NVR_REQUIRE(loss_dev && state_dev, NVR_EINVAL, "NULL loss or state");
    NVR_TRY(prepare(ctx, s, fields, nets));
    return enqueue_fwd(ctx, s, fields, b, nets, state_dev, loss_dev, C_out, D_out, hs(stream));
}

extern "C" nvr_status nvr_train_step_bwd(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                                         const nvr_batch *b, nvr_train_state *state_dev,
                                         nvr_stream stream) {
    clear_error();
    Net nets[2];
    NVR_TRY(step_check(ctx, s, fields, b, nets));
    NVR_REQUIRE(state_dev, NVR_EINVAL, "NULL state");
    for (int k = 0; k < s->n_fields; ++k)
        NVR_REQUIRE(ctx->ws[k].block && ctx->ws[k].cap >= s->max_samples, NVR_EINVAL,
                    "nvr_train_step_fwd was not run with this configuration");
    NVR_HIP(hipSetDevice(ctx->device));
    return enqueue_bwd(ctx, s, fields, b, nets, state_dev, hs(stream));
}

extern "C" nvr_status nvr_train_step(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                                     const nvr_batch *b, nvr_train_state *state_dev, float *loss_dev,
                                     nvr_stream stream) {
    clear_error();
    Net nets[2];
    NVR_TRY(step_check(ctx, s, fields, b, nets));
    NVR_REQUIRE(loss_dev && state_dev, NVR_EINVAL, "NULL loss or state");
    NVR_TRY(prepare(ctx, s, fields, nets));
    hipStream_t st = hs(stream);
    if ((ctx->flags & NVR_AUTOTUNE) && !deterministic(ctx) && s->precision == NVR_BF16) {
        bool need = false;
        for (int k = 0; k < s->n_fields; ++k) need |= !ctx->ws[k].tuned;
        if (need) {
            NVR_TRY(autotune(ctx, s, fields, b, nets, state_dev, loss_dev, st));
            // graphs captured with the old shapes
            for (auto &g : ctx->graphs) {
                if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
                if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
            }
            ctx->graphs.clear();
        }
    }
    if (!(ctx->flags & NVR_USE_GRAPH)) {
        NVR_TRY(enqueue_fwd(ctx, s, fields, b, nets, state_dev, loss_dev, nullptr, nullptr, st));
        return enqueue_bwd(ctx, s, fields, b, nets, state_dev, st);
    }
    const std::string key = graph_key(s, fields, b, state_dev, loss_dev);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        GraphEntry ge;
        NVR_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        nvr_status r1 = enqueue_fwd(ctx, s, fields, b, nets, state_dev, loss_dev, nullptr, nullptr,
                                    ctx->capture);
        nvr_status r2 = r1 == NVR_OK ? enqueue_bwd(ctx, s, fields, b, nets, state_dev, ctx->capture) : r1;
        hipError_t e = hipStreamEndCapture(ctx->capture, &ge.graph);
        if (r2 != NVR_OK) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            return r2;
        }
        if (e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            return NVR_EHIP;
        }
        NVR_HIP(hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
        it = ctx->graphs.emplace(key, ge).first;
    }
    NVR_HIP(hipGraphLaunch(it->second.exec, st));
    return NVR_OK;
}

extern "C" nvr_status nvr_launch_shape(const nvr_ctx *ctx, int32_t field, int32_t *shape) {
    clear_error();
    NVR_REQUIRE(ctx && shape && (field == 0 || field == 1), NVR_EINVAL, "bad arguments");
    const FieldWs &w = ctx->ws[field];
    shape[0] = w.enc_chunks;
    shape[1] = w.mlp_fwd_blocks;
    shape[2] = w.mlp_bwd_blocks;
    shape[3] = w.emit_chunks;
    shape[4] = ctx->comp_blocks;
    shape[5] = w.tuned ? 1 : 0;
    shape[6] = w.emit_block;
    return NVR_OK;
}

extern "C" nvr_status nvr_last_sample_count(nvr_ctx *ctx, int32_t field, int64_t *count,
                                            nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(ctx && count && (field == 0 || field == 1), NVR_EINVAL, "bad arguments");
    NVR_REQUIRE(ctx->ws[field].block, NVR_EINVAL, "field %d has no workspace yet", field);
    int32_t v = 0;
    NVR_HIP(hipMemcpyAsync(&v, ctx->ws[field].n_dev, sizeof(int32_t), hipMemcpyDeviceToHost,
                           hs(stream)));
    NVR_HIP(hipStreamSynchronize(hs(stream)));
    *count = v;
    return NVR_OK;
}

extern "C" nvr_status nvr_render(nvr_ctx *ctx, const nvr_step_desc *s, nvr_field *const *fields,
                                 int64_t n_rays, const float *o, const float *d, float t_stop,
                                 float *rgb, float *depth, nvr_stream stream) {
    clear_error();
    NVR_REQUIRE(ctx && s && fields && o && d && rgb && depth, NVR_EINVAL, "NULL argument");
    NVR_REQUIRE(n_rays >= 0 && n_rays < (1ll << 31), NVR_EINVAL, "n_rays out of range");
    NVR_REQUIRE(t_stop >= 0.f && t_stop < 1.f, NVR_EINVAL, "t_stop out of [0,1)");
    NVR_REQUIRE(s->n_fields == 1 || s->n_fields == 2, NVR_EINVAL, "n_fields must be 1 or 2");
    NVR_REQUIRE(s->max_samples >= 1, NVR_EINVAL, "max_samples < 1");
    if (n_rays == 0) return NVR_OK;
    Net nets[2];
    nvr_step_desc sd = *s;
    for (int k = 0; k < s->n_fields; ++k) {
        NVR_REQUIRE(fields[k] != nullptr, NVR_EINVAL, "field is NULL");
        nvr_field tmp = *fields[k];
        tmp.ray_begin = 0;
        tmp.ray_end = 0;
        sd.n_rays = n_rays;
        NVR_TRY(field_check(&tmp, &sd, &nets[k]));
    }
    hipStream_t st = hs(stream);
    NVR_HIP(hipSetDevice(ctx->device));
    // chunk the rays so that every ray's worst case fits the sample capacity
    int max_steps = 1;
    for (int k = 0; k < s->n_fields; ++k)
        max_steps = fields[k]->march.max_steps > max_steps ? fields[k]->march.max_steps : max_steps;
    int64_t chunk = s->max_samples / max_steps;
    if (chunk < 1) chunk = 1;
    if (chunk > n_rays) chunk = n_rays;
    for (int k = 0; k < s->n_fields; ++k)
        NVR_TRY(ensure_ws(ctx, k, fields[k], nets[k], s->precision, chunk, chunk * max_steps, false));
    for (int64_t r0 = 0; r0 < n_rays; r0 += chunk) {
        const int64_t nr = (n_rays - r0) < chunk ? (n_rays - r0) : chunk;
        for (int k = 0; k < s->n_fields; ++k)
            NVR_TRY(field_forward(ctx, k, fields[k], nets[k], s->precision, nr, 0, nr, o + 3 * r0,
                                  d + 3 * r0, /*train=*/false, st));
        const nvr_samples a = samples_of(ctx->ws[0]);
        nvr_samples bb;
        if (s->n_fields == 2) bb = samples_of(ctx->ws[1]);
        NVR_TRY(launch_composite_fwd(nr, a, s->n_fields == 2 ? &bb : nullptr, t_stop, rgb + 3 * r0,
                                     depth + r0, nullptr, st));
    }
    return NVR_OK;
}

// ---------------------------------------------------------------- networks
extern "C" size_t nvr_mlp_workspace(const nvr_mlp_desc *m, nvr_dtype math, int64_t n) {
    Net net;
    if (build_net(m, &net) != NVR_OK || n < 0) return 0;
    if (math == NVR_BF16 || math == NVR_F16) return mfma_ws_bytes(net, n);
    return plain_workspace(net, n);
}

static nvr_status mlp_args(const nvr_mlp_desc *m, int64_t n, const void *feat, nvr_dtype feat_dtype,
                           const float *dirs, const void *params, nvr_dtype math, Net *net) {
    NVR_TRY(build_net(m, net));
    NVR_REQUIRE(n >= 0 && n < (1ll << 31), NVR_EINVAL, "n out of range");
    if (math == NVR_BF16 || math == NVR_F16) {
        NVR_TRY(mfma_check(*net));
        NVR_REQUIRE(feat_dtype == math, NVR_EINVAL, "MFMA networks take features of the math type");
    } else {
        NVR_REQUIRE(math == NVR_F32, NVR_EINVAL, "math must be F32, F16 or BF16");
        NVR_REQUIRE(feat_dtype == NVR_F32, NVR_EINVAL, "f32 networks take f32 features");
    }
    if (n > 0) NVR_REQUIRE(feat && dirs && params, NVR_EINVAL, "NULL array");
    return NVR_OK;
}

extern "C" nvr_status nvr_mlp_fwd(const nvr_mlp_desc *m, int64_t n, const int32_t *n_dev,
                                  const void *feat, nvr_dtype feat_dtype, const float *dirs,
                                  const int32_t *ray_id, const void *params, nvr_dtype math,
                                  float *sigma, float *rgb, nvr_stream stream) {
    clear_error();
    Net net;
    NVR_TRY(mlp_args(m, n, feat, feat_dtype, dirs, params, math, &net));
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(sigma && rgb, NVR_EINVAL, "NULL output");
    hipStream_t st = hs(stream);
    if (math == NVR_BF16 || math == NVR_F16)
        return mfma_fwd(net, n, n_dev, n, (const uint16_t *)feat, false, dirs, ray_id, params,
                        math == NVR_F16, sigma, rgb, st);
    // the plain forward stores activations: use a transient workspace
    float *ws = nullptr;
    NVR_HIP(hipMallocAsync((void **)&ws, plain_workspace(net, n), st));
    PlainView F{(float *)feat, 1, net.n_in};
    nvr_status r = plain_fwd(net, n, n_dev, n, F, dirs, ray_id, (const float *)params, sigma, rgb, ws, st);
    NVR_HIP(hipFreeAsync(ws, st));
    return r;
}

extern "C" nvr_status nvr_mlp_bwd(const nvr_mlp_desc *m, int64_t n, const int32_t *n_dev,
                                  const void *feat, nvr_dtype feat_dtype, const float *dirs,
                                  const int32_t *ray_id, const void *params, nvr_dtype math,
                                  const float *dsigma, const float *drgb, float *dparams,
                                  float *dfeat, void *workspace, nvr_stream stream) {
    clear_error();
    Net net;
    NVR_TRY(mlp_args(m, n, feat, feat_dtype, dirs, params, math, &net));
    if (n == 0) return NVR_OK;
    NVR_REQUIRE(dsigma && drgb && dparams && workspace, NVR_EINVAL, "NULL array");
    hipStream_t st = hs(stream);
    if (math == NVR_BF16 || math == NVR_F16)
        return mfma_bwd(net, n, n_dev, n, (const uint16_t *)feat, false, dirs, ray_id, params,
                        math == NVR_F16, dsigma, drgb, dparams, dfeat, workspace, st);
    // plain: recompute the forward into the workspace, then back-propagate
    float *sig = nullptr;
    NVR_HIP(hipMallocAsync((void **)&sig, sizeof(float) * 4 * (size_t)n, st));
    float *rgb = sig + n;
    PlainView F{(float *)feat, 1, net.n_in};
    PlainView dF{dfeat, 1, net.n_in};
    nvr_status r = plain_fwd(net, n, n_dev, n, F, dirs, ray_id, (const float *)params, sig, rgb,
                             (float *)workspace, st);
    if (r == NVR_OK)
        r = plain_bwd(net, n, n_dev, n, F, (const float *)params, sig, rgb, dsigma, drgb, dparams, dF,
                      dfeat != nullptr, (float *)workspace, st);
    NVR_HIP(hipFreeAsync(sig, st));
    return r;
}
