"""Radiance-field state on the device and the whole-step driver.

A ``Field`` owns one field's parameter masters, their fp16 / bf16 copies,
gradients and Adam moments (device tensors); a ``Trainer`` owns an nvr
context and calls the library's fused training step and renderer.  Only
argument marshalling happens here.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from . import ops
from ._lib import call


class Deform:
    """Residual deformation network of a warped field (Sec. 4.2): its grid,
    pose, fp32 masters, gradients and Adam moments on the device."""

    def __init__(self, grid, theta, table, params, device="cuda"):
        self.grid = grid
        n_e = grid.n_entries
        self.theta = torch.as_tensor(np.asarray(theta, np.float32)).reshape(72).to(device)
        self.table = torch.as_tensor(np.asarray(table, np.float32)).reshape(n_e, 2).to(device)
        self.table_half = self.table.to(torch.float16)
        self.params = torch.as_tensor(np.asarray(params, np.float32)).reshape(-1).to(device)
        assert self.params.numel() == L.lib().nvr_deform_param_count()
        self.table_grad = torch.zeros_like(self.table)
        self.params_grad = torch.zeros_like(self.params)
        self.table_m = torch.zeros_like(self.table)
        self.table_v = torch.zeros_like(self.table)
        self.params_m = torch.zeros_like(self.params)
        self.params_v = torch.zeros_like(self.params)
        self.theta_grad = torch.zeros_like(self.theta)
        self._c = None

    def c(self):
        d = L.DeformState()
        d.grid = self.grid
        for k in ("theta", "table", "table_half", "params", "table_grad", "params_grad", "table_m",
                  "table_v", "params_m", "params_v", "theta_grad"):
            setattr(d, k, getattr(self, k).data_ptr())
        self._c = d            # kept alive while the field struct points at it
        return d


class Field:
    def __init__(self, work, fcfg, table, params, occ_words=None, rig=None, warp_desc=None,
                 ray_range=None, device="cuda", deform=None):
        self.work, self.fcfg = work, fcfg
        self.grid = ops.grid_desc_of(fcfg)
        self.mlp = ops.mlp_desc_of(fcfg)
        self.march = ops.march_desc_of(work, fcfg)
        n_e = self.grid.n_entries
        table = torch.as_tensor(np.asarray(table, np.float32)).reshape(n_e, 2)
        params = torch.as_tensor(np.asarray(params, np.float32)).reshape(-1)
        assert params.numel() == ops.mlp_param_count(self.mlp)
        self.table = table.to(device).contiguous()
        self.params = params.to(device).contiguous()
        self.table_half = self.table.to(torch.float16)
        self.params_bf16 = self.params.to(torch.bfloat16)
        self.table_grad = torch.zeros_like(self.table)
        self.params_grad = torch.zeros_like(self.params)
        self.table_m = torch.zeros_like(self.table)
        self.table_v = torch.zeros_like(self.table)
        self.params_m = torch.zeros_like(self.params)
        self.params_v = torch.zeros_like(self.params)
        self.occ = None
        if occ_words is not None and fcfg.occ_res > 0:
            self.occ = torch.from_numpy(np.asarray(occ_words, np.uint32).view(np.int32)).to(device)
        self.rig = rig
        self.warp = warp_desc
        self.node_dq_grad = self.bones_grad = None
        if rig is not None:
            self.node_dq_grad = torch.zeros_like(rig.node_dq)
            self.bones_grad = torch.zeros_like(rig.bones)
        self.ray_range = ray_range
        assert deform is None or rig is not None, "the deformation network needs the warp"
        self.deform = deform

    def c(self, n_rays):
        f = L.Field()
        f.grid, f.mlp, f.march = self.grid, self.mlp, self.march
        lo, hi = self.ray_range if self.ray_range is not None else (0, n_rays)
        f.ray_begin, f.ray_end = lo, hi
        p = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        f.occ = p(self.occ)
        f.table, f.table_half = p(self.table), p(self.table_half)
        f.params, f.params_bf16 = p(self.params), p(self.params_bf16)
        f.table_grad, f.params_grad = p(self.table_grad), p(self.params_grad)
        f.table_m, f.table_v = p(self.table_m), p(self.table_v)
        f.params_m, f.params_v = p(self.params_m), p(self.params_v)
        if self.rig is not None:
            f.has_warp = 1
            f.warp = self.warp
            f.rig = self.rig.c()
            f.node_dq_grad, f.bones_grad = p(self.node_dq_grad), p(self.bones_grad)
        if self.deform is not None:
            f.deform = C.pointer(self.deform.c())
        return f


def occupancy_update(field, precision, cells, points, grid, bits, decay=0.95,
                     tau_max=0.01 * 1024 / 3 ** 0.5):
    """One occupancy-grid update of `field` (a Field without warp): decays the
    density grid, takes the maximum with the field's density at the probes
    (cells [m] int32, points [m][3] float32), and rebuilds the bitfield
    `bits` from tau = min(tau_max, mean).  Returns tau (a 1-element tensor)."""
    m = int(cells.shape[0])
    cf = field.c(0)
    nb = L.lib().nvr_occupancy_workspace(C.byref(cf), precision, m)
    if nb == 0:
        call("nvr_occupancy_update", C.byref(cf), precision, m, None, None, 0.0, 0.0, None, None,
             None, None, None)   # raises with the library's reason
    ws = torch.empty(nb, dtype=torch.uint8, device=grid.device)
    tau = torch.empty(1, dtype=torch.float32, device=grid.device)
    p = lambda t: None if t is None or t.numel() == 0 else t.data_ptr()  # noqa: E731
    call("nvr_occupancy_update", C.byref(cf), precision, m, p(cells), p(points), decay, tau_max,
         grid.data_ptr(), bits.data_ptr(), tau.data_ptr(), ws.data_ptr(), ops._stream())
    return tau


class Trainer:
    """Owns an nvr context; runs training steps and renders."""

    def __init__(self, fields, n_rays, max_samples, precision=L.NVR_F32, lambda_depth=0.0,
                 adam=None, use_graph=False, loss_scale=1.0, device_index=0, autotune=False,
                 deterministic=False):
        self.fields = list(fields)
        self.n_rays = n_rays
        ctx = C.c_void_p()
        flags = ((L.NVR_USE_GRAPH if use_graph else 0) | (L.NVR_AUTOTUNE if autotune else 0) |
                 (L.NVR_DETERMINISTIC if deterministic else 0))
        call("nvr_create", C.byref(ctx), device_index, flags)
        self.ctx = ctx
        self.desc = L.StepDesc(len(self.fields), precision, n_rays, max_samples, lambda_depth,
                               adam or ops.adam_desc(), 1)
        self._cf = [f.c(n_rays) for f in self.fields]
        self._arr = (C.POINTER(L.Field) * len(self._cf))(*[C.pointer(f) for f in self._cf])
        self.state = ops.new_state(loss_scale)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.batch = None

    def set_batch(self, o, d, C_t, D_t=None, mask=None):
        self._batch_tensors = (o, d, C_t, D_t, mask)
        p = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        self.batch = L.Batch(p(o), p(d), p(C_t), p(D_t), p(mask))

    def step(self):
        call("nvr_train_step", self.ctx, C.byref(self.desc), self._arr, C.byref(self.batch),
             ops._p(self.state), ops._p(self.loss), ops._stream())
        return self.loss

    def forward(self, C_out=None, D_out=None):
        call("nvr_train_step_fwd", self.ctx, C.byref(self.desc), self._arr, C.byref(self.batch),
             ops._p(self.state), ops._p(self.loss), ops._p(C_out), ops._p(D_out), ops._stream())
        return self.loss

    def backward(self, apply_update=True):
        self.desc.apply_update = 1 if apply_update else 0
        try:
            call("nvr_train_step_bwd", self.ctx, C.byref(self.desc), self._arr,
                 C.byref(self.batch), ops._p(self.state), ops._stream())
        finally:
            self.desc.apply_update = 1

    def launch_shape(self, field=0):
        """Launch shapes in use for `field` (gather chunks, network forward and
        backward workgroups, emit chunks, compositing workgroups, tuned flag,
        emit samples per chunk)."""
        out = (C.c_int32 * 7)()
        call("nvr_launch_shape", self.ctx, field, out)
        return list(out)

    def sample_count(self, field=0):
        n = C.c_int64()
        call("nvr_last_sample_count", self.ctx, field, C.byref(n), ops._stream())
        return n.value

    def render(self, o, d, t_stop=1e-4):
        n = o.shape[0]
        rgb = torch.empty((n, 3), dtype=torch.float32, device=o.device)
        depth = torch.empty(n, dtype=torch.float32, device=o.device)
        call("nvr_render", self.ctx, C.byref(self.desc), self._arr, n, ops._p(o), ops._p(d),
             t_stop, ops._p(rgb), ops._p(depth), ops._stream())
        return rgb, depth

    def close(self):
        if self.ctx:
            L.lib().nvr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
