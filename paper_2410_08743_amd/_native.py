"""ctypes binding of libgsp.so (include/gsp.h).  Argument marshalling only.

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsp.so")

GSP_OK, GSP_EINVAL, GSP_ECAPACITY, GSP_ENOMEM, GSP_EHIP, GSP_EUNSUPPORTED = range(6)
GSP_ACCUMULATE = 1
GSP_POSE_SE3, GSP_POSE_T_SO3 = 0, 1
GSP_MAX_VIEWS = 32

# Every symbol include/gsp.h declares.
EXPORTS = (
    "gsp_create", "gsp_destroy", "gsp_workspace_size", "gsp_render_fwd", "gsp_render_bwd",
    "gsp_instances", "gsp_loss_l1", "gsp_loss_l1_scratch_bytes", "gsp_pose_adam",
    "gsp_inspect", "gsp_status_string", "gsp_last_error", "gsp_version",
    "gsp_profile_enable", "gsp_profile_read", "gsp_loss_rgb", "gsp_loss_rgb_scratch_bytes",
    "gsp_gaussian_adam", "gsp_gaussian_adam_scratch_bytes", "gsp_unproject_count",
    "gsp_unproject_scratch_bytes", "gsp_unproject", "gsp_loss_masked_l1",
    "gsp_loss_masked_l1_scratch_bytes", "gsp_loss_l1_noalloc", "gsp_render_fwd_store",
    "gsp_render_fwd_l1",
    "gsp_render_bwd_stored", "gsp_lists_bytes", "gsp_list_pairs", "gsp_twist_apply",
    "gsp_twist_chain", "gsp_render_bwd_pose_step",
)


class GspError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(message)
        self.status = status


class NativeLibraryMissing(RuntimeError):
    pass


class Gaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32)]


class View(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("roi_x", ctypes.c_int32), ("roi_y", ctypes.c_int32),
                ("roi_w", ctypes.c_int32), ("roi_h", ctypes.c_int32),
                ("bg", ctypes.c_float * 3)]


class Grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("pose", ctypes.c_void_p)]


class AdamParams(ctypes.Structure):
    _fields_ = [("lr_start", ctypes.c_float), ("lr_end", ctypes.c_float),
                ("total_steps", ctypes.c_int32), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("parametrization", ctypes.c_int32)]


class GaussianParams(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("logit_opacities", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class GaussianAdamParams(ctypes.Structure):
    _fields_ = [("lr_means_start", ctypes.c_double), ("lr_means_end", ctypes.c_double),
                ("total_steps", ctypes.c_int32), ("lr_sh_dc", ctypes.c_double),
                ("lr_sh_rest", ctypes.c_double), ("lr_opacities", ctypes.c_double),
                ("lr_scales", ctypes.c_double), ("lr_quats", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("aniso_r", ctypes.c_double), ("aniso_weight", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises NativeLibraryMissing when it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NativeLibraryMissing(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "gsp_create": ([ctypes.c_int, ctypes.POINTER(P)], I32),
        "gsp_destroy": ([P], I32),
        "gsp_workspace_size": ([I64, I32, I32, P, I64, ctypes.POINTER(SZ)], I32),
        "gsp_render_fwd": ([P, P, I32, P, P, P, P, P, SZ, I64, P], I32),
        "gsp_render_bwd": ([P, P, I32, P, P, P, P, SZ, I64, P, ctypes.c_uint32, P], I32),
        "gsp_instances": ([P, P, P, ctypes.POINTER(I64), ctypes.POINTER(I32)], I32),
        "gsp_loss_l1": ([P, I32, P, P, P, P, P, P, P], I32),
        "gsp_loss_l1_scratch_bytes": ([I32, P], SZ),
        "gsp_loss_l1_noalloc": ([P, I32, P, P, P, P, P, P], I32),
        "gsp_pose_adam": ([P, I32, P, P, P, P, P, P, P, P], I32),
        "gsp_inspect": ([P, P, I32, P, P, SZ, I64, ctypes.c_char_p, ctypes.POINTER(P),
                         ctypes.POINTER(I64)], I32),
        "gsp_profile_enable": ([P, ctypes.c_int], I32),
        "gsp_profile_read": ([P, I32, P, P, P, ctypes.POINTER(I32)], I32),
        "gsp_loss_rgb": ([P, I32, P, P, P, P, P, ctypes.c_float, P, SZ, P], I32),
        "gsp_loss_rgb_scratch_bytes": ([I32, P], SZ),
        "gsp_gaussian_adam": ([P, I64, I32, P, P, P, P, I32, P, P, P, P, P, P, P], I32),
        "gsp_gaussian_adam_scratch_bytes": ([I64], SZ),
        "gsp_unproject_count": ([P, I32, ctypes.POINTER(I64)], I32),
        "gsp_unproject_scratch_bytes": ([P, I32], SZ),
        "gsp_unproject": ([P, P, P, P, I32, ctypes.c_float, I32, P, P, SZ, P], I32),
        "gsp_loss_masked_l1": ([P, I32, P, P, P, P, P, P, P, P], I32),
        "gsp_loss_masked_l1_scratch_bytes": ([I32, P], SZ),
        "gsp_render_fwd_store": ([P, P, I32, P, P, P, P, P, SZ, I64, P, SZ, I64, P], I32),
        "gsp_render_fwd_l1": ([P, P, I32, P, P, P, P, P, P, P, SZ, I64, P], I32),
        "gsp_render_bwd_stored": ([P, P, I32, P, P, P, P, SZ, I64, P, SZ, I64, P, ctypes.c_uint32,
                                   P], I32),
        "gsp_lists_bytes": ([I32, P, I64], SZ),
        "gsp_list_pairs": ([P, P, P, ctypes.POINTER(I64), ctypes.POINTER(I32)], I32),
        "gsp_twist_apply": ([P, I32, P, P, P, P], I32),
        "gsp_twist_chain": ([P, I32, P, P, P, P], I32),
        "gsp_render_bwd_pose_step": ([P, P, I32, P, P, P, P, SZ, I64, P, P, P, P, P, P], I32),
        "gsp_status_string": ([I32], ctypes.c_char_p),
        "gsp_last_error": ([], ctypes.c_char_p),
        "gsp_version": ([], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(status, what=""):
    if status != GSP_OK:
        L = lib()
        msg = f"{what}: {L.gsp_status_string(status).decode()}: {L.gsp_last_error().decode()}"
        raise GspError(status, msg)


def make_view(cam):
    roi = cam.roi if getattr(cam, "roi", None) is not None else (0, 0, cam.width, cam.height)
    bg = getattr(cam, "bg", None) or (0.0, 0.0, 0.0)
    return View(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                float(cam.cy), int(roi[0]), int(roi[1]), int(roi[2]), int(roi[3]),
                (ctypes.c_float * 3)(*[float(b) for b in bg]))


def ptr_array(ptrs):
    """Host array of device pointers (None for NULL entries)."""
    return (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])


def view_array(cams):
    arr = (View * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = make_view(c)
    return arr
