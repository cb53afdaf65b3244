"""ctypes mirror of include/pgsag.h and the loader of libpgsag.so.

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly when the library is missing; there is no fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgsag.so")

ABI_VERSION = 3
NUM_STAGES = 8
STAGES = ("tile_mask", "preprocess", "depth_sort", "emit", "tile_sort", "composite",
          "backward_composite", "backward_preprocess")

OK, INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, UNSUPPORTED, HIP_ERROR = range(5)


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class Outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("normal", C.c_void_p), ("dist", C.c_void_p),
                ("depth", C.c_void_p), ("alpha", C.c_void_p), ("n_contrib", C.c_void_p)]


class GradOutputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("normal", C.c_void_p), ("dist", C.c_void_p),
                ("depth", C.c_void_p), ("alpha", C.c_void_p), ("count", C.c_void_p)]


class Render(C.Structure):
    _fields_ = [("set", C.c_int32), ("reserved", C.c_int32), ("cam", Camera), ("mask", C.c_void_p),
                ("out", Outputs), ("gout", GradOutputs)]


class Config(C.Structure):
    _fields_ = [("tile", C.c_int32), ("persistent", C.c_int32), ("queue_chunk", C.c_int32),
                ("workgroups_per_cu", C.c_int32), ("alpha_min", C.c_float), ("t_min", C.c_float),
                ("alpha_max", C.c_float), ("dilation", C.c_float), ("z_near", C.c_float),
                ("fov_clamp", C.c_float), ("logit_min", C.c_float), ("depth_guard", C.c_float),
                ("bg", C.c_float * 3), ("bwd_reduce", C.c_int32),
                ("deterministic", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("workspace_bytes", C.c_uint64), ("desc_bytes", C.c_uint64), ("n_records", C.c_uint64),
                ("n_tiles", C.c_uint64), ("n_pixels", C.c_uint64), ("pair_capacity", C.c_uint64),
                ("tile_bits", C.c_int32), ("reserved", C.c_int32)]


class Layout(C.Structure):
    _fields_ = [(name, C.c_uint64) for name in
                ("status", "tile_count", "sat", "ranges", "queue", "records", "depth_key", "rect",
                 "n_active", "pair_tile", "pair_record", "pixel_T", "pixel_last", "grad2d", "work", "end")]


class LossConfig(C.Structure):
    _fields_ = [("lambda_rgb", C.c_float), ("lambda_normal", C.c_float), ("boundary_weight", C.c_float),
                ("lambda_load", C.c_float), ("normal_norm", C.c_int32), ("normal_eps", C.c_float),
                ("load_term", C.c_int32), ("reserved", C.c_int32)]


class AdamConfig(C.Structure):
    _fields_ = [("lr", C.c_float), ("b1", C.c_float), ("b2", C.c_float), ("eps", C.c_float),
                ("step_state", C.c_void_p), ("m_offset", C.c_int64), ("v_offset", C.c_int64),
                ("write_grads", C.c_int32), ("reserved", C.c_int32)]


class VoteView(C.Structure):
    _fields_ = [("cam", Camera), ("mask", C.c_void_p)]


class Volume(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("voxel", C.c_float), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("trunc", C.c_float)]


class DepthView(C.Structure):
    _fields_ = [("cam", Camera), ("depth", C.c_void_p)]


class Status(C.Structure):
    _fields_ = [("pairs_needed", C.c_uint64), ("overflow", C.c_uint32), ("n_visible", C.c_uint32),
                ("error", C.c_uint32), ("reserved", C.c_uint32)]


SYMBOLS = ("pgsag_version", "pgsag_last_error", "pgsag_default_config", "pgsag_plan", "pgsag_pack",
           "pgsag_layout_of", "pgsag_forward", "pgsag_backward", "pgsag_binning",
           "pgsag_read_status", "pgsag_adam_step", "pgsag_load_stats", "pgsag_default_loss_config",
           "pgsag_loss", "pgsag_luminance_weights", "pgsag_adam_step_device", "pgsag_backward_adam",
           "pgsag_vote", "pgsag_dbscan_workspace", "pgsag_dbscan", "pgsag_dbscan_static", "pgsag_group_views",
           "pgsag_fuse_depth", "pgsag_tsdf_integrate")

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libpgsag.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_2501_01677_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float
    L.pgsag_version.restype = C.c_int
    L.pgsag_last_error.restype = C.c_char_p
    L.pgsag_default_config.argtypes = [C.POINTER(Config)]
    L.pgsag_default_config.restype = None
    L.pgsag_plan.argtypes = [C.POINTER(Config), C.POINTER(Gaussians), i32, C.POINTER(Render), i32, u64,
                             C.POINTER(PlanInfo)]
    L.pgsag_pack.argtypes = [C.POINTER(Config), C.POINTER(Gaussians), C.POINTER(Grads), i32,
                             C.POINTER(Render), i32, u64, vp, C.c_size_t]
    L.pgsag_layout_of.argtypes = [vp, C.POINTER(Layout)]
    for f in (L.pgsag_forward, L.pgsag_backward):
        f.argtypes = [vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.pgsag_binning.argtypes = [vp, vp, vp, C.c_size_t, vp]
    L.pgsag_read_status.argtypes = [vp, vp, C.POINTER(Status), vp]
    L.pgsag_adam_step.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
    L.pgsag_adam_step_device.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, vp, vp]
    L.pgsag_backward_adam.argtypes = [vp, vp, vp, C.c_size_t, C.POINTER(AdamConfig), vp, C.POINTER(vp)]
    L.pgsag_load_stats.argtypes = [vp, vp, vp, C.POINTER(vp), vp, vp]
    L.pgsag_default_loss_config.argtypes = [C.POINTER(LossConfig)]
    L.pgsag_default_loss_config.restype = None
    L.pgsag_loss.argtypes = [C.POINTER(LossConfig), vp, vp, vp, u64, C.POINTER(vp), C.POINTER(vp), vp, vp]
    L.pgsag_luminance_weights.argtypes = [vp, vp, vp, u64, i32, vp, vp, vp]
    L.pgsag_vote.argtypes = [C.POINTER(VoteView), vp, i32, vp, i64, f32, i32, vp, vp, vp, vp]
    L.pgsag_dbscan_workspace.argtypes = [i64, C.POINTER(C.c_uint64)]
    L.pgsag_dbscan.argtypes = [vp, i64, vp, C.c_uint32, f32, i32, vp, vp, vp, vp, vp, u64, vp]
    L.pgsag_dbscan_static.argtypes = [vp, i64, vp, C.c_uint32, f32, i32, vp, vp, vp, vp, vp]
    L.pgsag_fuse_depth.argtypes = [C.POINTER(vp), i32, i32, i32, vp, vp, vp]
    L.pgsag_tsdf_integrate.argtypes = [C.POINTER(Volume), C.POINTER(DepthView), vp, i32, f32, vp, vp, i32, vp]
    L.pgsag_group_views.argtypes = [C.POINTER(VoteView), vp, i32, vp, i64, vp, i32, f32, C.c_uint32, vp, vp, vp]
    for name in SYMBOLS:
        if name not in ("pgsag_last_error", "pgsag_default_config", "pgsag_default_loss_config"):
            getattr(L, name).restype = C.c_int
    if L.pgsag_version() != ABI_VERSION:
        raise RuntimeError("libpgsag.so ABI version mismatch")
    _lib = L
    return L


class PgsagError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().pgsag_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def check(code, where):
    if code != OK:
        raise PgsagError(code, where)
