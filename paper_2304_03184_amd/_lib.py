"""ctypes binding of libnvr.so (argument marshalling only).

Every structure mirrors include/nvr.h field for field.  Loading fails loudly
when the library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnvr.so")

i32, i64, f32, vp = C.c_int32, C.c_int64, C.c_float, C.c_void_p

NVR_OK, NVR_EINVAL, NVR_EUNSUPPORTED, NVR_EHIP, NVR_ENOMEM, NVR_ENONFINITE, NVR_EOVERFLOW = \
    0, -1, -2, -3, -4, -5, -6
NVR_F32, NVR_F16, NVR_BF16 = 0, 1, 2
NVR_USE_GRAPH = 1
NVR_AUTOTUNE = 2
NVR_DETERMINISTIC = 4
MAX_LEVELS = 32


class GridDesc(C.Structure):
    _fields_ = [("n_levels", i32), ("n_features", i32), ("log2_table", i32),
                ("res", i32 * MAX_LEVELS), ("dense", i32 * MAX_LEVELS),
                ("offset", i64 * (MAX_LEVELS + 1)),
                ("aabb_min", f32 * 3), ("aabb_max", f32 * 3)]

    @property
    def n_entries(self) -> int:
        return int(self.offset[self.n_levels])


class MarchDesc(C.Structure):
    _fields_ = [("aabb_min", f32 * 3), ("aabb_max", f32 * 3), ("near_t", f32), ("far_t", f32),
                ("step", f32), ("max_steps", i32), ("occ_res", i32)]


class WarpDesc(C.Structure):
    _fields_ = [("n_joints", i32), ("k_joints", i32), ("sigma_skin", f32), ("n_nodes", i32),
                ("k_nodes", i32), ("n_frames", i32), ("r_node", f32), ("lut_res", i32),
                ("lut_min", f32 * 3), ("lut_max", f32 * 3)]


class WarpRig(C.Structure):
    _fields_ = [("joints", vp), ("bones", vp), ("node_dq", vp), ("node_pos", vp), ("lut", vp)]


class LutDesc(C.Structure):
    _fields_ = [("canon_min", f32 * 3), ("canon_max", f32 * 3), ("live_min", f32 * 3),
                ("live_max", f32 * 3), ("canon_res", i32), ("live_res", i32), ("k_nodes", i32),
                ("n_nodes", i32), ("r_ed", f32)]


NVR_POOL_REJECT, NVR_POOL_FIRST, NVR_POOL_APPEND, NVR_POOL_REPLACE = 0, 1, 2, 3


class MlpDesc(C.Structure):
    _fields_ = [("n_in", i32), ("n_density_hidden", i32), ("density_hidden", i32 * 4),
                ("density_out", i32), ("sh_degree", i32), ("n_colour_hidden", i32),
                ("colour_hidden", i32 * 4)]


class Samples(C.Structure):
    _fields_ = [("off", vp), ("sigma", vp), ("rgb", vp), ("t", vp), ("dt", vp)]


class TrainState(C.Structure):
    _fields_ = [("step", i32), ("finite", i32), ("loss_scale", f32), ("pad", f32)]


class AdamDesc(C.Structure):
    _fields_ = [("lr", f32), ("beta1", f32), ("beta2", f32), ("eps", f32), ("lr_decay", f32)]


class DeformState(C.Structure):
    _fields_ = [("grid", GridDesc), ("theta", vp), ("table", vp), ("table_half", vp), ("params", vp),
                ("table_grad", vp), ("params_grad", vp), ("table_m", vp), ("table_v", vp),
                ("params_m", vp), ("params_v", vp), ("theta_grad", vp)]


class Field(C.Structure):
    _fields_ = [("grid", GridDesc), ("mlp", MlpDesc), ("march", MarchDesc), ("has_warp", i32),
                ("warp", WarpDesc), ("rig", WarpRig), ("ray_begin", i64), ("ray_end", i64),
                ("occ", vp), ("table", vp), ("table_half", vp), ("params", vp),
                ("params_bf16", vp), ("table_grad", vp), ("params_grad", vp), ("table_m", vp),
                ("table_v", vp), ("params_m", vp), ("params_v", vp), ("node_dq_grad", vp),
                ("bones_grad", vp), ("deform", C.POINTER(DeformState))]


class StepDesc(C.Structure):
    _fields_ = [("n_fields", i32), ("precision", i32), ("n_rays", i64), ("max_samples", i64),
                ("lambda_depth", f32), ("adam", AdamDesc), ("apply_update", i32)]


class Batch(C.Structure):
    _fields_ = [("o", vp), ("d", vp), ("C_t", vp), ("D_t", vp), ("mask", vp)]


P = C.POINTER
_SIGS = {
    "nvr_last_error": (C.c_char_p, []),
    "nvr_version": (C.c_char_p, []),
    "nvr_grid_init": (i32, [P(GridDesc), i32, i32, i32, i32, i32, P(f32), P(f32)]),
    "nvr_encode_fwd": (i32, [P(GridDesc), i64, vp, vp, i32, vp, i32, vp]),
    "nvr_encode_bwd": (i32, [P(GridDesc), i64, vp, vp, i32, vp, vp, vp, vp]),
    "nvr_encode_bwd_workspace": (C.c_size_t, [P(GridDesc), i64]),
    "nvr_encode_bwd_binned": (i32, [P(GridDesc), i64, vp, vp, vp, vp, vp, vp, vp]),
    "nvr_encode_bwd_deterministic_workspace": (C.c_size_t, [P(GridDesc), i64]),
    "nvr_encode_bwd_deterministic": (i32, [P(GridDesc), i64, vp, vp, vp, vp, vp, vp, vp]),
    "nvr_encode_fwd_grouped": (i32, [P(GridDesc), i64, vp, vp, vp, vp]),
    "nvr_encode_bwd_binned_grouped": (i32, [P(GridDesc), i64, vp, vp, vp, vp, vp, vp, vp]),
    "nvr_occupancy_workspace": (C.c_size_t, [P(Field), i32, i64]),
    "nvr_occupancy_update": (i32, [P(Field), i32, i64, vp, vp, f32, f32, vp, vp, vp, vp, vp]),
    "nvr_live_lut": (i32, [P(LutDesc), vp, vp, vp, vp, vp]),
    "nvr_deform_workspace": (C.c_size_t, [P(GridDesc), i64]),
    "nvr_deform_param_count": (i64, []),
    "nvr_deform_fwd": (i32, [P(GridDesc), i64, vp, vp, vp, vp, i32, vp, vp, vp]),
    "nvr_deform_bwd": (i32, [P(GridDesc), i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]),
    "nvr_visibility": (i32, [i32, i32, vp, vp, vp, i32, i32, f32, vp, vp]),
    "nvr_human_distance": (i32, [i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, f32, f32, vp, vp,
                                 vp]),
    "nvr_object_distance": (i32, [i32, vp, vp, vp, i32, f32, f32, vp, vp]),
    "nvr_pool_step": (i32, [P(i32), P(i32), i32, P(f32), i32, f32, P(i32), P(i32)]),
    "nvr_pool_select": (i32, [i32, P(f32), i32, P(i32), P(i32)]),
    "nvr_depth_assemble": (i32, [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "nvr_probe_gather": (i32, [vp, C.c_size_t, i64, i32, C.c_uint32, vp, vp]),
    "nvr_march_workspace": (C.c_size_t, [i64]),
    "nvr_march": (i32, [P(MarchDesc), i64, i64, i64, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp,
                        vp, vp]),
    "nvr_march_noalloc": (i32, [P(MarchDesc), i64, i64, i64, vp, vp, vp, i64, vp, vp, vp, vp,
                                vp, vp, vp]),
    "nvr_warp_fwd": (i32, [P(WarpDesc), P(WarpRig), i64, vp, vp, vp, vp, vp]),
    "nvr_warp_bwd": (i32, [P(WarpDesc), P(WarpRig), i64, vp, vp, vp, vp, i32, vp, vp, vp, vp]),
    "nvr_mlp_param_count": (i32, [P(MlpDesc), P(i64)]),
    "nvr_mlp_fwd": (i32, [P(MlpDesc), i64, vp, vp, i32, vp, vp, vp, i32, vp, vp, vp]),
    "nvr_mlp_workspace": (C.c_size_t, [P(MlpDesc), i32, i64]),
    "nvr_mlp_bwd": (i32, [P(MlpDesc), i64, vp, vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp,
                          vp]),
    "nvr_composite_fwd": (i32, [i64, P(Samples), P(Samples), f32, vp, vp, vp, vp]),
    "nvr_composite_bwd": (i32, [i64, P(Samples), P(Samples), vp, vp, vp, vp, vp, vp, vp, vp,
                                vp]),
    "nvr_loss": (i32, [i64, vp, vp, vp, vp, vp, f32, vp, vp, vp, vp, vp]),
    "nvr_state_begin": (i32, [vp, vp]),
    "nvr_check_finite": (i32, [i64, vp, vp, vp]),
    "nvr_adam": (i32, [P(AdamDesc), i64, vp, vp, vp, vp, i32, vp, vp, i32, vp]),
    "nvr_state_end": (i32, [vp, vp]),
    "nvr_create": (i32, [P(vp), i32, C.c_uint32]),
    "nvr_destroy": (None, [vp]),
    "nvr_train_step_fwd": (i32, [vp, P(StepDesc), P(P(Field)), P(Batch), vp, vp, vp, vp, vp]),
    "nvr_train_step_bwd": (i32, [vp, P(StepDesc), P(P(Field)), P(Batch), vp, vp]),
    "nvr_train_step": (i32, [vp, P(StepDesc), P(P(Field)), P(Batch), vp, vp, vp]),
    "nvr_launch_shape": (i32, [vp, i32, P(i32)]),
    "nvr_last_sample_count": (i32, [vp, i32, P(i64), vp]),
    "nvr_render": (i32, [vp, P(StepDesc), P(P(Field)), i64, vp, vp, f32, vp, vp, vp]),
}


class NvrError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises ImportError if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return sorted(_SIGS)


def call(name, *args):
    """Calls an entry point returning nvr_status; raises NvrError on failure."""
    rc = getattr(lib(), name)(*args)
    if rc != NVR_OK:
        raise NvrError(name, rc, lib().nvr_last_error().decode())
    return rc
