"""ctypes mirror of include/sdirt.h and the loader of libsdirt.so.

Argument marshalling only: the structs below are byte-for-byte copies of the
C declarations.  Loading fails loudly when the library has not been built.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdirt.so")

OK, EINVAL, EUNSUPPORTED, ELAUNCH, ENODEVICE, ESCRATCH = 0, -1, -2, -3, -4, -5
NOALLOC_SCRATCH_BYTES = 16 << 20
SPHERE, PLANE, STOP, ASPHERE, IDEAL = 0, 1, 2, 3, 4
MAT_CAUCHY, MAT_ABBE = 0, 1
DP_SIGMOID, DP_MICROLENS = 0, 1
SPLAT_BOX, SPLAT_TENT = 0, 1
NORM_NONE, NORM_SUM, NORM_MAX = 0, 1, 2
F32, F64, BF16 = 0, 1, 2
SRC_DENSE, SRC_BANK, SRC_BANK2D = 0, 1, 2
BANK_FP32, BANK_SPLIT_BF16 = 0, 1
LOSS_L2MAX, LOSS_KL = 0, 1
MAX_SURFACES = 24


class Surface(C.Structure):
    _fields_ = [("kind", C.c_int), ("material", C.c_int),
                ("mat_p0", C.c_double), ("mat_p1", C.c_double),
                ("c", C.c_double), ("t", C.c_double),
                ("semi_diameter", C.c_double), ("conic", C.c_double),
                ("asph", C.c_double * 5), ("focal", C.c_double)]


class Lens(C.Structure):
    _fields_ = [("n_surfaces", C.c_int), ("stop", C.c_int),
                ("surfaces", C.POINTER(Surface)),
                ("object_material", C.c_int),
                ("object_p0", C.c_double), ("object_p1", C.c_double),
                ("f_number", C.c_double), ("focus_depth", C.c_double),
                ("ref_wavelength", C.c_double)]


class LensInfo(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("efl", "bfd", "sensor_distance", "stop_radius", "z_ep",
                 "rho_ep", "m_num", "sensor_z")]


class Sensor(C.Structure):
    _fields_ = [("pitch", C.c_double), ("dp_mode", C.c_int),
                ("sigmoid_k", C.c_double), ("ml_h", C.c_double),
                ("ml_f", C.c_double), ("ml_w", C.c_double), ("ml_r", C.c_double)]


class PsfQuery(C.Structure):
    _fields_ = [("n_fields", C.c_int), ("n_depths", C.c_int),
                ("n_wavelengths", C.c_int),
                ("fields", C.POINTER(C.c_double)),
                ("depths", C.POINTER(C.c_double)),
                ("wavelengths", C.POINTER(C.c_double)),
                ("n_points", C.c_int), ("points", C.c_void_p),
                ("rays_x", C.c_int), ("rays_y", C.c_int), ("seed", C.c_uint32),
                ("jitter", C.c_int), ("ks", C.c_int), ("splat", C.c_int),
                ("normalize", C.c_int), ("out_dtype", C.c_int), ("math", C.c_int),
                ("deterministic", C.c_int)]


class RenderDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("C", C.c_int), ("H", C.c_int), ("W", C.c_int),
                ("ks", C.c_int), ("source", C.c_int), ("psf_channels", C.c_int),
                ("psf_dtype", C.c_int), ("bank_fields", C.c_int),
                ("bank_depths", C.c_int), ("bank_lambdas", C.c_int),
                ("field_radii", C.POINTER(C.c_double)),
                ("inv_depths", C.POINTER(C.c_double)),
                ("lambda_of_channel", C.c_int * 4), ("pitch", C.c_double),
                ("bank_fields_y", C.c_int), ("field_y", C.POINTER(C.c_double)),
                ("bank_math", C.c_int)]


class MlpDesc(C.Structure):
    _fields_ = [("n_hidden", C.c_int), ("width", C.c_int), ("n_out", C.c_int),
                ("n_freq", C.c_int),
                ("x_half", C.c_double), ("y_half", C.c_double),
                ("iv_lo", C.c_double), ("iv_hi", C.c_double),
                ("lam_lo", C.c_double), ("lam_hi", C.c_double), ("loss", C.c_int)]


class MlpRenderDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("C", C.c_int), ("H", C.c_int), ("W", C.c_int),
                ("ks", C.c_int), ("pitch", C.c_double), ("wavelength", C.c_double * 4)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "sdirt_version": (C.c_int, []),
    "sdirt_status_string": (C.c_char_p, [C.c_int]),
    "sdirt_resolve_lens": (C.c_int, [C.POINTER(Lens), C.POINTER(LensInfo)]),
    "sdirt_pupil": (C.c_int, [C.POINTER(Lens), C.c_double, C.POINTER(C.c_double),
                              C.POINTER(C.c_double)]),
    "sdirt_n_params": (C.c_int, [C.POINTER(Lens)]),
    "sdirt_trace_rays": (C.c_int, [C.POINTER(Lens), C.c_double, C.c_int, C.c_int,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "sdirt_trace_dp_psf": (C.c_int, [C.POINTER(Lens), C.POINTER(Sensor),
                                     C.POINTER(PsfQuery), C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "sdirt_trace_dp_psf_chunks": (C.c_int, [C.POINTER(Lens), C.POINTER(Sensor),
                                            C.POINTER(PsfQuery), C.c_void_p,
                                            C.c_void_p, C.c_int, C.c_void_p]),
    "sdirt_trace_dp_psf_backward": (C.c_int, [C.POINTER(Lens), C.POINTER(Sensor),
                                              C.POINTER(PsfQuery), C.c_void_p,
                                              C.c_void_p, C.c_void_p]),
    "sdirt_render_dp": (C.c_int, [C.POINTER(RenderDesc), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdirt_render_dp_backward": (C.c_int, [C.POINTER(RenderDesc), C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "sdirt_render_dp_psf_backward": (C.c_int, [C.POINTER(RenderDesc), C.c_void_p, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdirt_mlp_n_params": (C.c_int, [C.POINTER(MlpDesc), C.POINTER(C.c_longlong)]),
    "sdirt_mlp_workspace_size": (C.c_int, [C.POINTER(MlpDesc), C.c_int,
                                           C.POINTER(C.c_size_t)]),
    "sdirt_mlp_forward": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_longlong,
                                    C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                    C.c_int, C.c_void_p]),
    "sdirt_mlp_forward_noalloc": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_longlong,
                                            C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "sdirt_mlp_render": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.POINTER(MlpRenderDesc),
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_void_p]),
    "sdirt_mlp_backward": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "sdirt_mlp_vjp": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_longlong, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                C.c_void_p]),
    "sdirt_mlp_adam": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_int, C.c_float, C.c_void_p]),
    "sdirt_mlp_train_step": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int, C.c_float, C.c_int, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    "sdirt_psf_hybrid": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.POINTER(Lens),
                                   C.POINTER(Sensor), C.POINTER(PsfQuery), C.c_int,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "sdirt_calib_fma64": (C.c_int, [C.c_longlong, C.c_int, C.c_void_p, C.c_void_p]),
    "sdirt_mlp_train": (C.c_int, [C.POINTER(MlpDesc), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int, C.c_int, C.c_float, C.c_float, C.c_int,
                                  C.c_int, C.c_longlong, C.c_void_p, C.c_void_p,
                                  C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libsdirt.so is not built (run python -m paper_2503_11213_amd.build)")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(l, name):
                fn = getattr(l, name)
                fn.restype = res
                fn.argtypes = args
        _lib = l
    return _lib


class SdirtError(RuntimeError):
    def __init__(self, fn, status):
        msg = lib().sdirt_status_string(status).decode()
        super().__init__("%s failed: %s (%d)" % (fn, msg, status))
        self.status = status


def check(fn, status):
    if status != OK:
        raise SdirtError(fn, status)
