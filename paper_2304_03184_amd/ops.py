"""Torch-facing wrappers of the nvr C ABI.

Each function only marshals arguments (device pointers of torch tensors, the
current HIP stream) into the corresponding entry point of libnvr.so; every
step of the computation runs in the library's kernels.  The autograd
Functions pair each forward entry point with its hand-written backward.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L
from ._lib import call

F32, F16, BF16 = L.NVR_F32, L.NVR_F16, L.NVR_BF16
_DT = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f3(v):
    return (C.c_float * 3)(*[float(a) for a in v])


def _dev(t, dtype=None):
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    if dtype is not None:
        assert t.dtype == dtype, f"expected {dtype}, got {t.dtype}"
    return t


# ---------------------------------------------------------------- descriptors
def grid_desc(n_levels, n_features, log2_table, res_min, res_max, aabb_min, aabb_max):
    g = L.GridDesc()
    call("nvr_grid_init", C.byref(g), n_levels, n_features, log2_table, res_min, res_max,
         _f3(aabb_min), _f3(aabb_max))
    return g


def grid_desc_of(fcfg):
    return grid_desc(fcfg.n_levels, fcfg.n_features, fcfg.log2_table, fcfg.res_min,
                     fcfg.res_max, fcfg.aabb_min, fcfg.aabb_max)


def march_desc(aabb_min, aabb_max, near=0.0, far=1e30, step=0.0, max_steps=128, occ_res=0):
    return L.MarchDesc(_f3(aabb_min), _f3(aabb_max), near, far, step, max_steps, occ_res)


def march_desc_of(work, fcfg):
    return march_desc(fcfg.aabb_min, fcfg.aabb_max, work.near, work.far, work.fixed_step,
                      work.max_steps, fcfg.occ_res)


def mlp_desc(n_in, density_hidden, density_out, sh_degree, colour_hidden):
    dh = (C.c_int32 * 4)(*density_hidden)
    ch = (C.c_int32 * 4)(*colour_hidden)
    return L.MlpDesc(n_in, len(density_hidden), dh, density_out, sh_degree, len(colour_hidden), ch)


def mlp_desc_of(fcfg):
    return mlp_desc(fcfg.enc_width, fcfg.density_hidden, fcfg.density_out, fcfg.sh_degree,
                    fcfg.colour_hidden)


def mlp_param_count(md):
    n = C.c_int64()
    call("nvr_mlp_param_count", C.byref(md), C.byref(n))
    return n.value


def warp_desc(n_joints=24, k_joints=4, sigma_skin=0.1, n_nodes=1024, k_nodes=8, n_frames=1,
              r_node=0.1, lut_res=128, lut_min=(-1.0,) * 3, lut_max=(1.0,) * 3):
    return L.WarpDesc(n_joints, k_joints, sigma_skin, n_nodes, k_nodes, n_frames, r_node,
                      lut_res, _f3(lut_min), _f3(lut_max))


class Rig:
    """Device copies of the warp inputs (joints, bones, node motions, look-up)."""

    def __init__(self, joints, bones, node_dq, node_pos, lut):
        self.joints, self.bones, self.node_dq, self.node_pos, self.lut = \
            joints, bones, node_dq, node_pos, lut

    @classmethod
    def from_numpy(cls, rig, device="cuda"):
        import numpy as np
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)  # noqa: E731
        lut = torch.from_numpy(np.ascontiguousarray(rig["knn"]).view(np.int16)).to(device)
        return cls(t(rig["joints"], torch.float32), t(rig["bones"], torch.float32),
                   t(rig["node_dq"], torch.float32), t(rig["node_pos"], torch.float32), lut)

    def c(self):
        return L.WarpRig(self.joints.data_ptr(), self.bones.data_ptr(), self.node_dq.data_ptr(),
                         self.node_pos.data_ptr(), self.lut.data_ptr())


# ---------------------------------------------------------------- encode
def encode_fwd(g, x, table, feat_dtype=torch.float32):
    _dev(x, torch.float32)
    _dev(table)
    n = x.shape[0]
    feat = torch.empty((n, g.n_levels * g.n_features), dtype=feat_dtype, device=x.device)
    call("nvr_encode_fwd", C.byref(g), n, _p(x), _p(table), _DT[table.dtype], _p(feat),
         _DT[feat_dtype], _stream())
    return feat


def encode_bwd(g, x, table, dfeat, dtable, dx=None):
    _dev(dfeat, torch.float32)
    _dev(dtable, torch.float32)
    call("nvr_encode_bwd", C.byref(g), x.shape[0], _p(x), _p(table), _DT[table.dtype],
         _p(dfeat), _p(dtable), _p(dx), _stream())


def encode_bwd_binned(g, x, table, dfeat, dtable, dx=None):
    """Binned (atomic-free per contribution) backward for a float16 table."""
    _dev(dfeat, torch.float32)
    _dev(dtable, torch.float32)
    n = x.shape[0]
    nb = L.lib().nvr_encode_bwd_workspace(C.byref(g), n)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=x.device)
    call("nvr_encode_bwd_binned", C.byref(g), n, _p(x), _p(table), _p(dfeat), _p(dtable),
         _p(dx), _p(ws), _stream())


def encode_bwd_deterministic(g, x, table, dfeat, dtable, dx=None):
    """encode_bwd_binned with every sum in an order fixed by the inputs
    (bit-identical results call to call)."""
    _dev(dfeat, torch.float32)
    _dev(dtable, torch.float32)
    n = x.shape[0]
    nb = L.lib().nvr_encode_bwd_deterministic_workspace(C.byref(g), n)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=x.device)
    call("nvr_encode_bwd_deterministic", C.byref(g), n, _p(x), _p(table), _p(dfeat),
         _p(dtable), _p(dx), _p(ws), _stream())


def grouped_width(g):
    """Features per sample in one level-group plane (2 x ceil(L / 8))."""
    return 2 * ((g.n_levels + 7) // 8)


def encode_fwd_grouped(g, x, table):
    """fp16 features in the level-group layout [8][n][2 lpg] from an fp16 table."""
    n = x.shape[0]
    feat = torch.empty((8, n, grouped_width(g)), dtype=torch.float16, device=x.device)
    call("nvr_encode_fwd_grouped", C.byref(g), n, _p(x), _p(table), _p(feat), _stream())
    return feat


def encode_bwd_binned_grouped(g, x, table, dfeat, dtable, dx=None):
    """Binned backward with float32 feature gradients in the level-group layout."""
    _dev(dfeat, torch.float32)
    _dev(dtable, torch.float32)
    n = x.shape[0]
    nb = L.lib().nvr_encode_bwd_workspace(C.byref(g), n)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=x.device)
    call("nvr_encode_bwd_binned_grouped", C.byref(g), n, _p(x), _p(table), _p(dfeat),
         _p(dtable), _p(dx), _p(ws), _stream())


def live_lut(knn, node_canon, node_dq, canon_box, canon_res, live_box, live_res, r_ed=0.1):
    """Live look-up table of the fast neighbour search (Sec. 4.2, Eq. 1): the
    canonical voxel index per live voxel, -1 for holes.  knn [canon_res^3][K]
    uint16 (int16 storage) node ids, node_canon [n][3], node_dq [n][8]; the boxes
    are (min xyz, max xyz) pairs."""
    assert knn.dtype == torch.int16 and knn.dim() == 2 and knn.shape[0] == canon_res ** 3
    assert node_canon.dtype == torch.float32 and node_dq.dtype == torch.float32
    assert node_canon.shape[0] == node_dq.shape[0]
    d = L.LutDesc()
    d.canon_min[:], d.canon_max[:] = canon_box[0], canon_box[1]
    d.live_min[:], d.live_max[:] = live_box[0], live_box[1]
    d.canon_res, d.live_res, d.k_nodes = canon_res, live_res, knn.shape[1]
    d.n_nodes, d.r_ed = node_canon.shape[0], r_ed
    knn, node_canon, node_dq = knn.contiguous(), node_canon.contiguous(), node_dq.contiguous()
    lut = torch.empty(live_res ** 3, dtype=torch.int32, device=knn.device)
    call("nvr_live_lut", C.byref(d), _p(knn), _p(node_canon), _p(node_dq), _p(lut), _stream())
    return lut


def _workspace(nbytes, device):
    # 256-byte aligned device bytes (torch's allocations are)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def deform_fwd(g, x, theta, table, params, math=F32):
    """Deformation network (Sec. 4.2): x + MLP([enc(x), theta]) for x [n][3];
    math F32 (float32 layers) or F16 (matrix-core kernels)."""
    n = x.shape[0]
    x, theta, table, params = (t.contiguous() for t in (x, theta, table, params))
    out = torch.empty_like(x)
    ws = _workspace(L.lib().nvr_deform_workspace(C.byref(g), n), x.device)
    call("nvr_deform_fwd", C.byref(g), n, _p(x), _p(theta), _p(table), _p(params), math,
         _p(out), _p(ws), _stream())
    return out


def deform_bwd(g, x, theta, table, params, dx_can, want_dx=True, want_dtheta=True, math=F32):
    """Gradients of sum(dx_can . deform_fwd(...)): (dparams, dtable, dx, dtheta)."""
    n = x.shape[0]
    x, theta, table, params, dx_can = (t.contiguous() for t in (x, theta, table, params, dx_can))
    dparams = torch.zeros_like(params)
    dtable = torch.zeros_like(table)
    dx = torch.zeros_like(x) if want_dx else None
    dtheta = torch.zeros_like(theta) if want_dtheta else None
    ws = _workspace(L.lib().nvr_deform_workspace(C.byref(g), n), x.device)
    call("nvr_deform_bwd", C.byref(g), n, _p(x), _p(theta), _p(table), _p(params), math,
         _p(dx_can), _p(dparams), _p(dtable), _p(dx), _p(dtheta), _p(ws), _stream())
    return dparams, dtable, dx, dtheta


def visibility(nodes, proj, depth, eps=0.01):
    """Eq. 5 visibility bits: nodes [F][M][3], proj [F][3][4], depth [F][H][W]
    (float32, device) -> int32 [F][ceil(M / 32)] words (uint32 bit patterns)."""
    F, M = nodes.shape[0], nodes.shape[1]
    H, W = depth.shape[1], depth.shape[2]
    assert nodes.dtype == proj.dtype == depth.dtype == torch.float32
    assert proj.shape == (F, 3, 4) and depth.shape[0] == F
    nodes, proj, depth = nodes.contiguous(), proj.contiguous(), depth.contiguous()
    bits = torch.empty((F, (M + 31) // 32), dtype=torch.int32, device=nodes.device)
    call("nvr_visibility", F, M, _p(nodes), _p(proj), _p(depth), H, W, eps, _p(bits), _stream())
    return bits


def human_distance(pool_theta, pool_bits, pool_t, q_theta, q_bits, q_t, beta, beta_vis=0.01,
                   beta_h=0.02):
    """Eq. 6 of a query frame against every pooled frame: (E [n] float32,
    xor counts [n] int32)."""
    n, n_pose = pool_theta.shape
    n_words = pool_bits.shape[1]
    args = [t.contiguous() for t in (pool_theta, pool_bits, pool_t, q_theta, q_bits, beta)]
    E = torch.empty(n, dtype=torch.float32, device=pool_theta.device)
    cnt = torch.empty(n, dtype=torch.int32, device=pool_theta.device)
    call("nvr_human_distance", n, n_pose, n_words, _p(args[0]), _p(args[1]), _p(args[2]),
         _p(args[3]), _p(args[4]), int(q_t), _p(args[5]), beta_vis, beta_h, _p(E), _p(cnt),
         _stream())
    return E, cnt


def object_distance(pool_d, pool_t, q_d, q_t, beta_d=1.0, beta_o=0.02):
    """Eq. 7 of a query frame against every pooled frame: E [n] float32."""
    n = pool_d.shape[0]
    a, b, c = pool_d.contiguous(), pool_t.contiguous(), q_d.contiguous()
    E = torch.empty(n, dtype=torch.float32, device=pool_d.device)
    call("nvr_object_distance", n, _p(a), _p(b), _p(c), int(q_t), beta_d, beta_o, _p(E),
         _stream())
    return E


def pool_step(pool, dist, frame, cap=100, gamma=2.5):
    """One spatial-pool decision on the host: pool (list of frame ids) is
    updated in place; returns (action, slot)."""
    buf = (C.c_int32 * cap)(*pool)
    n = C.c_int32(len(pool))
    d = (C.c_float * max(len(pool), 1))(*[float(x) for x in dist])
    act, slot = C.c_int32(), C.c_int32()
    call("nvr_pool_step", buf, C.byref(n), cap, d, frame, gamma, C.byref(act), C.byref(slot))
    pool[:] = list(buf[:n.value])
    return act.value, slot.value


def pool_select(dist, m=10):
    """Slots of the m smallest distances (ties by slot), host side."""
    n = len(dist)
    d = (C.c_float * max(n, 1))(*[float(x) for x in dist])
    out = (C.c_int32 * max(min(m, n), 1))()
    k = C.c_int32()
    call("nvr_pool_select", n, d, m, out, C.byref(k))
    return list(out[:k.value])


def depth_assemble(rgb_a, depth_a, alpha_a, rgb_b, depth_b, alpha_b):
    """Per-pixel depth test of two renderings: (rgb [n][3], depth [n])."""
    n = depth_a.shape[0]
    ins = [t.contiguous().float() for t in (rgb_a, depth_a, alpha_a, rgb_b, depth_b, alpha_b)]
    rgb = torch.empty((n, 3), dtype=torch.float32, device=depth_a.device)
    depth = torch.empty(n, dtype=torch.float32, device=depth_a.device)
    call("nvr_depth_assemble", n, *[_p(t) for t in ins], _p(rgb), _p(depth), _stream())
    return rgb, depth


def probe_gather(table, n, loads, seed=1):
    """Random 16-byte gathers over `table`'s bytes split into eight slices
    (measurement probe, not part of the method); returns the [8][n] xors."""
    out = torch.empty((8, n), dtype=torch.int32, device=table.device)
    call("nvr_probe_gather", _p(table), table.numel() * table.element_size(), n, loads, seed,
         _p(out), _stream())
    return out


class EncodeFn(torch.autograd.Function):
    """feat = encode(x, table); backward scatters into the table gradient and
    (when x requires grad) accumulates the position gradient."""

    @staticmethod
    def forward(ctx, x, table, g):
        ctx.g = g
        ctx.save_for_backward(x, table)
        return encode_fwd(g, x.contiguous(), table.contiguous(), torch.float32)

    @staticmethod
    def backward(ctx, dfeat):
        x, table = ctx.saved_tensors
        dtable = torch.zeros(table.shape, dtype=torch.float32, device=table.device)
        dx = torch.zeros_like(x) if ctx.needs_input_grad[0] else None
        encode_bwd(ctx.g, x, table, dfeat.contiguous().float(), dtable, dx)
        return dx, dtable.to(table.dtype), None


# ---------------------------------------------------------------- march
def march(md, o, d, occ=None, capacity=None, ray_begin=0, ray_end=None, sync=True):
    n_rays = o.shape[0]
    ray_end = n_rays if ray_end is None else ray_end
    cap = n_rays * md.max_steps if capacity is None else capacity
    dev = o.device
    off = torch.empty(n_rays + 1, dtype=torch.int32, device=dev)
    ray_id = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    t = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    dt = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    x = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
    n_dev = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(L.lib().nvr_march_workspace(n_rays), 4), dtype=torch.uint8, device=dev)
    call("nvr_march", C.byref(md), n_rays, ray_begin, ray_end, _p(o), _p(d), _p(occ), cap,
         _p(off), _p(ray_id), _p(t), _p(dt), _p(x), _p(n_dev), _p(ws), _stream())
    out = dict(off=off, ray_id=ray_id, t=t, dt=dt, x=x, n_dev=n_dev, capacity=cap)
    if sync:
        n = int(n_dev.item())
        if n > cap:
            raise L.NvrError("nvr_march", L.NVR_EOVERFLOW, f"{n} samples > capacity {cap}")
        for k in ("ray_id", "t", "dt", "x"):
            out[k] = out[k][:n]
        out["n"] = n
    return out


# ---------------------------------------------------------------- warp
def warp_fwd(wd, rig, x, n_dev=None):
    xc = torch.empty_like(x)
    call("nvr_warp_fwd", C.byref(wd), C.byref(rig.c()), x.shape[0], _p(n_dev), _p(x), None,
         _p(xc), _stream())
    return xc


def warp_bwd(wd, rig, x, dxc, d_node_dq, d_bones=None, n_parts=1, dx_live=None):
    call("nvr_warp_bwd", C.byref(wd), C.byref(rig.c()), x.shape[0], None, _p(x), None,
         _p(dxc), n_parts, _p(d_node_dq), _p(d_bones), _p(dx_live), _stream())


class WarpFn(torch.autograd.Function):
    """x_can = warp(x_live; node_dq, bones) with the joints, node positions and
    look-up table of `rig`; backward to the live positions, node motions and
    bones."""

    @staticmethod
    def forward(ctx, x, node_dq, bones, wd, rig):
        r = Rig(rig.joints, bones.contiguous(), node_dq.contiguous(), rig.node_pos, rig.lut)
        ctx.wd, ctx.r = wd, r
        x = x.contiguous()
        ctx.save_for_backward(x)
        return warp_fwd(wd, r, x)

    @staticmethod
    def backward(ctx, dxc):
        (x,) = ctx.saved_tensors
        r = ctx.r
        d_dq = torch.zeros_like(r.node_dq)
        d_b = torch.zeros_like(r.bones)
        dx = torch.zeros_like(x) if ctx.needs_input_grad[0] else None
        warp_bwd(ctx.wd, r, x, dxc.contiguous(), d_dq, d_b, dx_live=dx)
        return dx, d_dq, d_b, None, None


# ---------------------------------------------------------------- networks
def mlp_fwd(md, feat, dirs, params, ray_id=None, math_dtype=F32):
    n = feat.shape[0]
    sigma = torch.empty(n, dtype=torch.float32, device=feat.device)
    rgb = torch.empty((n, 3), dtype=torch.float32, device=feat.device)
    call("nvr_mlp_fwd", C.byref(md), n, None, _p(feat), _DT[feat.dtype], _p(dirs), _p(ray_id),
         _p(params), math_dtype, _p(sigma), _p(rgb), _stream())
    return sigma, rgb


def mlp_bwd(md, feat, dirs, params, dsigma, drgb, dparams, ray_id=None, math_dtype=F32,
            want_dfeat=True):
    n = feat.shape[0]
    dfeat = torch.empty((n, md.n_in), dtype=torch.float32, device=feat.device) \
        if want_dfeat else None
    ws = torch.empty(max(L.lib().nvr_mlp_workspace(C.byref(md), math_dtype, n), 4),
                     dtype=torch.uint8, device=feat.device)
    call("nvr_mlp_bwd", C.byref(md), n, None, _p(feat), _DT[feat.dtype], _p(dirs), _p(ray_id),
         _p(params), math_dtype, _p(dsigma), _p(drgb), _p(dparams), _p(dfeat), _p(ws), _stream())
    return dfeat


class FieldNetFn(torch.autograd.Function):
    """(sigma, rgb) = networks(feat, dirs); backward recomputes the forward."""

    @staticmethod
    def forward(ctx, feat, params, dirs, ray_id, md, math_dtype):
        ctx.md, ctx.math = md, math_dtype
        ctx.save_for_backward(feat, params, dirs, ray_id)
        return mlp_fwd(md, feat, dirs, params, ray_id, math_dtype)

    @staticmethod
    def backward(ctx, dsigma, drgb):
        feat, params, dirs, ray_id = ctx.saved_tensors
        dparams = torch.zeros(params.shape, dtype=torch.float32, device=params.device)
        dfeat = mlp_bwd(ctx.md, feat, dirs, params, dsigma.contiguous(), drgb.contiguous(),
                        dparams, ray_id, ctx.math)
        return dfeat.to(feat.dtype), dparams.to(params.dtype), None, None, None, None


# ---------------------------------------------------------------- compositing
def samples(off, sigma, rgb, t, dt):
    return L.Samples(off.data_ptr(), sigma.data_ptr(), rgb.data_ptr(), t.data_ptr(),
                     dt.data_ptr())


def composite_fwd(a, b=None, n_rays=None, t_stop=0.0, device="cuda"):
    C_ = torch.empty((n_rays, 3), dtype=torch.float32, device=device)
    D = torch.empty(n_rays, dtype=torch.float32, device=device)
    TN = torch.empty(n_rays, dtype=torch.float32, device=device)
    call("nvr_composite_fwd", n_rays, C.byref(a), C.byref(b) if b is not None else None,
         t_stop, _p(C_), _p(D), _p(TN), _stream())
    return C_, D, TN


def composite_bwd(a, na, C_, D, dC, dD, b=None, nb=0, device="cuda"):
    n_rays = C_.shape[0]
    dsa = torch.empty(max(na, 1), dtype=torch.float32, device=device)
    dra = torch.empty((max(na, 1), 3), dtype=torch.float32, device=device)
    dsb = drb = None
    if b is not None:
        dsb = torch.empty(max(nb, 1), dtype=torch.float32, device=device)
        drb = torch.empty((max(nb, 1), 3), dtype=torch.float32, device=device)
    call("nvr_composite_bwd", n_rays, C.byref(a), C.byref(b) if b is not None else None,
         _p(C_), _p(D), _p(dC), _p(dD), _p(dsa), _p(dra), _p(dsb), _p(drb), _stream())
    return dsa[:na], dra[:na], (dsb[:nb] if dsb is not None else None), \
        (drb[:nb] if drb is not None else None)


class CompositeFn(torch.autograd.Function):
    """(C, D) = composite(sigma, rgb) of one ray-major sample list."""

    @staticmethod
    def forward(ctx, sigma, rgb, t, dt, off):
        a = samples(off, sigma, rgb, t, dt)
        C_, D, _ = composite_fwd(a, n_rays=off.shape[0] - 1, device=sigma.device)
        ctx.save_for_backward(sigma, rgb, t, dt, off, C_, D)
        return C_, D

    @staticmethod
    def backward(ctx, dC, dD):
        sigma, rgb, t, dt, off, C_, D = ctx.saved_tensors
        a = samples(off, sigma, rgb, t, dt)
        dsig, drgb, _, _ = composite_bwd(a, sigma.shape[0], C_, D, dC.contiguous(),
                                         dD.contiguous(), device=sigma.device)
        return dsig, drgb, None, None, None


# ---------------------------------------------------------------- loss / Adam
def loss(C_, D, C_t, D_t=None, mask=None, lambda_d=0.0, loss_scale=None):
    n = C_.shape[0]
    out = torch.empty(1, dtype=torch.float32, device=C_.device)
    dC = torch.empty_like(C_)
    dD = torch.empty_like(D)
    call("nvr_loss", n, _p(C_), _p(D), _p(C_t), _p(D_t), _p(mask), lambda_d, _p(loss_scale),
         _p(out), _p(dC), _p(dD), _stream())
    return out, dC, dD


def adam_desc(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, lr_decay=1.0):
    return L.AdamDesc(lr, beta1, beta2, eps, lr_decay)


def new_state(loss_scale=1.0, device="cuda"):
    """Device-resident nvr_train_state: int32 step, int32 finite, f32 scale, pad."""
    s = torch.zeros(4, dtype=torch.int32, device=device)
    s.view(torch.float32)[2] = loss_scale
    s[1] = 1
    return s


def state_values(state):
    s = state.cpu()
    return dict(step=int(s[0]), finite=int(s[1]), loss_scale=float(s.view(torch.float32)[2]))


def adam(ad, param, m, v, grad, state, skip_zero=False, copy=None):
    call("nvr_adam", C.byref(ad), param.numel(), _p(param), _p(m), _p(v), _p(grad),
         1 if skip_zero else 0, _p(state), _p(copy), _DT[copy.dtype] if copy is not None else 0,
         _stream())


def state_begin(state):
    call("nvr_state_begin", _p(state), _stream())


def check_finite(g, state):
    call("nvr_check_finite", g.numel(), _p(g), _p(state), _stream())


def state_end(state):
    call("nvr_state_end", _p(state), _stream())
