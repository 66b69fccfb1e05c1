"""ctypes mirror of include/memgs.h and loader of the in-tree libmemgs.so.

Argument marshalling only: every step of the path runs in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmemgs.so")

MGS_OK = 0
MGS_ERR_INVALID_ARG = -1
MGS_ERR_WORKSPACE = -2
MGS_ERR_HIP = -3
MGS_ERR_TOO_LARGE = -4
MGS_ERR_SCRATCH = -5
MGS_LOSS_SCRATCH_BYTES = 64 << 20   # fixed scratch of mgs_mapping_loss_noalloc, per GPU
MGS_LOSS_NOALLOC_MAX_VIEWS = 64


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opac", C.c_void_p), ("sh", C.c_void_p), ("sh_degree", C.c_int32), ("reserved", C.c_int32)]


class GaussianGrads(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opac", C.c_void_p), ("d_sh", C.c_void_p), ("grad_norm_sum", C.c_void_p),
                ("visible_count", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("Tcw", C.c_float * 12), ("near_z", C.c_float),
                ("map", C.c_int32)]


class RenderOpts(C.Structure):
    _fields_ = [("bg_rgb", C.c_float * 3), ("bg_depth", C.c_float), ("need_backward", C.c_int32),
                ("count_blended", C.c_int32), ("stage_ms", C.POINTER(C.c_float)),
                ("stage_events", C.POINTER(C.c_void_p))]


class ForwardInfo(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_visible", C.c_int64), ("n_instances", C.c_int64),
                ("n_bins", C.c_int64), ("n_pixels", C.c_int64), ("ws_required", C.c_size_t),
                ("off_pair_depth", C.c_size_t), ("off_pair_rect", C.c_size_t), ("off_pair_uvr", C.c_size_t),
                ("off_rank_pair", C.c_size_t), ("off_inst_key", C.c_size_t), ("off_inst_rec", C.c_size_t),
                ("off_bin_range", C.c_size_t), ("off_n_contrib", C.c_size_t), ("off_n_blend", C.c_size_t),
                ("n_views", C.c_int32),
                ("n_maps", C.c_int32), ("need_backward", C.c_int32), ("bin_tx", C.c_int32),
                ("bin_ty", C.c_int32), ("inst_bin_bits", C.c_int32), ("inst_rank_bits", C.c_int32)]


class LossOpts(C.Structure):
    _fields_ = [("lambda_ssim", C.c_float), ("w_depth", C.c_float), ("w_iso", C.c_float), ("reserved", C.c_int32)]


class PgOpts(C.Structure):
    _fields_ = [("patch", C.c_int32), ("min_keypoints", C.c_int32), ("samples", C.c_int32),
                ("opacity", C.c_float), ("scale_factor", C.c_float), ("reserved", C.c_int32)]


class AdamOpts(C.Structure):
    _fields_ = [("lr", C.c_float * 5), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32)]


class GaussiansOut(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opac", C.c_void_p),
                ("sh", C.c_void_p)]


EXPORTS = ("mgs_render_forward", "mgs_render_backward", "mgs_voxel_merge", "mgs_merge_mask", "mgs_mapping_loss",
           "mgs_mapping_loss_noalloc", "mgs_patch_grid_sample", "mgs_adam_step", "mgs_status_string", "mgs_last_hip_error", "mgs_abi_version")

_lib = None


class MemgsError(RuntimeError):
    def __init__(self, fn: str, status: int):
        lib = load()
        msg = lib.mgs_status_string(status).decode()
        if status == MGS_ERR_HIP:
            msg += ": " + lib.mgs_last_hip_error().decode()
        super().__init__(f"{fn} failed ({status}): {msg}")
        self.status = status


def load():
    """Load libmemgs.so (built by paper_2509_13536_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_13536_amd.build` "
                           "(the HIP library is required; there is no fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.mgs_render_forward.restype = C.c_int32
    L.mgs_render_forward.argtypes = [C.POINTER(Gaussians), C.c_int32, C.POINTER(Camera), C.c_int32,
                                     C.POINTER(RenderOpts), P, C.c_size_t, C.POINTER(ForwardInfo), P, P, P, P]
    L.mgs_render_backward.restype = C.c_int32
    L.mgs_render_backward.argtypes = [C.POINTER(Gaussians), C.c_int32, C.POINTER(Camera), C.c_int32,
                                      C.POINTER(RenderOpts), C.POINTER(ForwardInfo), P, C.c_size_t, P, P, P,
                                      C.POINTER(GaussianGrads), P, P]
    L.mgs_voxel_merge.restype = C.c_int32
    L.mgs_voxel_merge.argtypes = [C.POINTER(Gaussians), P, C.c_float, C.c_float, C.c_int32,
                                  C.POINTER(GaussiansOut), P, P, P, C.c_size_t, C.POINTER(C.c_size_t),
                                  C.POINTER(C.c_int64), P]
    L.mgs_merge_mask.restype = C.c_int32
    L.mgs_merge_mask.argtypes = [P, P, P, C.c_int64, C.c_float, C.c_int32, C.c_int32, P, P]
    L.mgs_mapping_loss.restype = C.c_int32
    L.mgs_mapping_loss.argtypes = [P, C.c_int32, P, P, P, P, P, C.c_int64, C.POINTER(LossOpts), P, C.c_size_t,
                                   C.POINTER(C.c_size_t), P, P, P, P, P]
    L.mgs_mapping_loss_noalloc.restype = C.c_int32
    L.mgs_mapping_loss_noalloc.argtypes = [P, C.c_int32, P, P, P, P, P, C.c_int64, C.POINTER(LossOpts),
                                           C.POINTER(C.c_size_t), P, P, P, P, P]
    L.mgs_patch_grid_sample.restype = C.c_int32
    L.mgs_patch_grid_sample.argtypes = [C.POINTER(Camera), P, P, C.c_int64, P, P, C.POINTER(PgOpts),
                                        C.POINTER(GaussiansOut), P, P, C.c_size_t, C.POINTER(C.c_size_t),
                                        C.POINTER(C.c_int64), P]
    L.mgs_adam_step.restype = C.c_int32
    L.mgs_adam_step.argtypes = [C.POINTER(GaussiansOut), C.c_int64, C.c_int32, C.POINTER(GaussianGrads),
                                C.POINTER(GaussiansOut), C.POINTER(GaussiansOut), C.POINTER(AdamOpts), P]
    L.mgs_status_string.restype = C.c_char_p
    L.mgs_status_string.argtypes = [C.c_int32]
    L.mgs_last_hip_error.restype = C.c_char_p
    L.mgs_last_hip_error.argtypes = []
    L.mgs_abi_version.restype = C.c_int32
    L.mgs_abi_version.argtypes = []
    _lib = L
    return L
