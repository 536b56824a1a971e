"""ctypes binding of ``liblbm.so`` (the C-ABI declared in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  Loading fails loudly when the library is missing.
"""
import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_ENAN = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_ESTATE",
               -5: "LBM_ENAN"}


class LbmConfig(C.Structure):
    """Mirror of ``lbm_config``."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("batch", C.c_int32),
        ("radius", C.c_double), ("tau", C.c_double), ("accel_z", C.c_double),
        ("n_modes", C.c_int32),
        ("kz", C.c_double), ("kappa", C.c_double), ("l0_frac", C.c_double), ("l_frac", C.c_double),
        ("period", C.c_double),
        ("force_off_step", C.c_int64),
        ("storage", C.c_int32), ("wall", C.c_int32), ("pattern", C.c_int32), ("init", C.c_int32),
        ("u_tau", C.c_double),
        ("adjoint", C.c_int32), ("block", C.c_int32), ("zchunk", C.c_int32), ("xcd_remap", C.c_int32),
        ("collision", C.c_int32), ("equilibrium", C.c_int32),
    ]


class LbmLayout(C.Structure):
    """Mirror of ``lbm_layout``."""
    _fields_ = [
        ("n_fluid_columns", C.c_int64), ("plane_pitch", C.c_int64), ("n_fluid_nodes", C.c_int64),
        ("state_bytes", C.c_int64), ("workspace_bytes", C.c_int64), ("bytes_per_update", C.c_int64),
        ("population_stride", C.c_int64), ("record_bytes", C.c_int64),
    ]


CONFIG_DEFAULTS = dict(nx=24, ny=24, nz=48, batch=1, radius=10.0, tau=0.8, accel_z=0.0, n_modes=0,
                       kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=1.0, force_off_step=0,
                       storage=0, wall=0, pattern=0, init=0, u_tau=0.0, adjoint=0, block=0, zchunk=0,
                       xcd_remap=0, collision=0, equilibrium=0)


def make_config(**kw) -> LbmConfig:
    """``lbm_config`` from keyword values (unknown keys are ignored)."""
    vals = {k: kw.get(k, v) for k, v in CONFIG_DEFAULTS.items()}
    return LbmConfig(**vals)


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


CHECKED_LIB_PATH = os.path.join(HERE, "liblbm_checked.so")
_libs = {}


def lib():
    """The loaded library (raises if ``liblbm.so`` has not been built)."""
    return load(LIB_PATH)


def checked_lib():
    """The checked build (device-side bounds tests, ``lbm_check_flags``),
    loaded beside the release library in its own namespace."""
    return load(CHECKED_LIB_PATH)


def load(path):
    """A library built from these sources at ``path``, with the signatures
    set (each path loaded once; ctypes loads it with local symbols, so two
    builds coexist in one process)."""
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run paper_2405_12082_amd/build.py)")
    L = C.CDLL(path)
    vp, i32, i64, dp, fp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double), C.c_void_p
    cfgp = C.POINTER(LbmConfig)
    sig = {
        "lbm_describe": ([cfgp, C.POINTER(LbmLayout)], C.c_int),
        "lbm_workspace_bytes": ([cfgp, C.POINTER(C.c_size_t)], C.c_int),
        "lbm_init": ([cfgp, dp, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
        "lbm_step": ([vp, i32], C.c_int),
        "lbm_step_graph": ([vp, i32, i32], C.c_int),
        "lbm_stream_copy": ([vp, i32], C.c_int),
        "lbm_step_persistent": ([vp, i32], C.c_int),
        "lbm_set_launch": ([vp, i32, i32, i32, i32, i32], C.c_int),
        "lbm_set_fused": ([vp, i32, i32, i32], C.c_int),
        "lbm_step_persistent_graph": ([vp, i32, i32], C.c_int),
        "lbm_get_step": ([vp, C.POINTER(i64)], C.c_int),
        "lbm_moments": ([vp, fp, fp], C.c_int),
        "lbm_populations": ([vp, fp], C.c_int),
        "lbm_set_populations": ([vp, fp, i64], C.c_int),
        "lbm_diagnostics": ([vp, dp], C.c_int),
        "lbm_set_watchdog": ([vp, C.c_double], C.c_int),
        "lbm_profile_accumulate": ([vp], C.c_int),
        "lbm_profile_reset": ([vp], C.c_int),
        "lbm_profile_read": ([vp, dp], C.c_int),
        "lbm_state_bytes": ([vp, C.POINTER(C.c_size_t)], C.c_int),
        "lbm_save": ([vp, vp, C.POINTER(i64)], C.c_int),
        "lbm_load": ([vp, vp, i64], C.c_int),
        "lbm_adjoint_reset": ([vp, i64, i64], C.c_int),
        "lbm_adjoint_step": ([vp, i32, vp, C.c_size_t, vp], C.c_int),
        "lbm_energy": ([vp, dp], C.c_int),
        "lbm_energy_accumulate": ([vp, vp], C.c_int),
        "lbm_recompute": ([vp, vp, i64, i32, vp, C.c_size_t], C.c_int),
        "lbm_recompute_moments": ([vp, vp, i64, i32, vp, C.c_size_t, vp, C.c_size_t], C.c_int),
        "lbm_adjoint_step_moments": ([vp, i32, vp, C.c_size_t, vp], C.c_int),
        "lbm_step_recording": ([vp, i32, vp, C.c_size_t], C.c_int),
        "lbm_ring_sample": ([vp, C.c_double, i32, vp], C.c_int),
        "lbm_ring_spectrum": ([vp, vp, i32, i32, vp, vp, vp], C.c_int),
        "lbm_ring_spectrum_static": ([vp, i32, i32, i32, i32, vp, vp, vp, vp], C.c_int),
        "lbm_check_flags": ([vp, C.POINTER(C.c_uint32), C.POINTER(i32)], C.c_int),
        "lbm_last_error": ([vp], C.c_char_p),
        "lbm_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _libs[path] = L
    return L


def header_functions():
    """Names of the functions declared in include/lbm.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def describe(cfg: LbmConfig) -> LbmLayout:
    out = LbmLayout()
    rc = lib().lbm_describe(C.byref(cfg), C.byref(out))
    if rc != LBM_OK:
        raise LbmError(rc, "invalid configuration")
    return out
