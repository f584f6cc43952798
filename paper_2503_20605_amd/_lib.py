"""ctypes binding of libiblb.so (the C ABI declared in include/iblb.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Importing this module fails loudly when the library has not been
built; there is no fallback of any kind."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiblb.so")

IBLB_OK = 0
IBLB_EINVAL = -1
IBLB_ENOMEM = -2
IBLB_EDEVICE = -3
IBLB_EUNSTABLE = -4
IBLB_ELIMIT = -5
IBLB_PERIODIC = 0
IBLB_WALL = 1
IBLB_F32 = 0
IBLB_F16 = 1
IBLB_BF16 = 2

STATUS_NAMES = {0: "IBLB_OK", -1: "IBLB_EINVAL", -2: "IBLB_ENOMEM", -3: "IBLB_EDEVICE",
                -4: "IBLB_EUNSTABLE", -5: "IBLB_ELIMIT"}

EXPORTED = (
    "iblb_workspace_bytes", "iblb_create", "iblb_destroy", "iblb_last_error",
    "iblb_set_interface", "iblb_init_rest", "iblb_init_fields", "iblb_write_populations",
    "iblb_read_populations", "iblb_set_force_field", "iblb_step", "iblb_read_fields",
    "iblb_read_nodes", "iblb_diagnostics", "iblb_set_lb_variant", "iblb_autotune",
    "iblb_set_graph_steps", "iblb_set_active", "iblb_set_timing", "iblb_last_timing", "iblb_time_lattice",
    "iblb_probe_copy", "iblb_run_to_rest", "iblb_set_viscosity_ratio", "iblb_inside_mask",
    "iblb_contact_radius", "iblb_set_membrane_shear", "iblb_set_node_respacing",
    "iblb_mlp_workspace_bytes", "iblb_mlp_create", "iblb_mlp_destroy", "iblb_mlp_last_error",
    "iblb_mlp_param_count", "iblb_mlp_set_params", "iblb_mlp_get_params", "iblb_mlp_forward",
    "iblb_mlp_gradients", "iblb_mlp_adam_step", "iblb_mlp_forward_noalloc",
)


class iblb_params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("bc", ctypes.c_int * 3), ("tau", ctypes.c_double),
                ("sigma", ctypes.c_double), ("theta_eq", ctypes.c_double),
                ("xi", ctypes.c_double), ("n_exp", ctypes.c_int), ("m_exp", ctypes.c_int),
                ("wetting", ctypes.c_int)]


class iblb_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass", ctypes.c_double),
                ("momentum", ctypes.c_double * 3), ("sum_phi", ctypes.c_double * 3),
                ("sum_F", ctypes.c_double * 3), ("dropped_F", ctypes.c_double * 3),
                ("volume", ctypes.c_double), ("area", ctypes.c_double),
                ("contact_radius", ctypes.c_double), ("height", ctypes.c_double),
                ("theta_meas", ctypes.c_double), ("max_normal_speed", ctypes.c_double),
                ("max_speed", ctypes.c_double), ("min_h", ctypes.c_double),
                ("edge_min", ctypes.c_double), ("edge_max", ctypes.c_double),
                ("status", ctypes.c_int32)]

    def to_dict(self, dim=3):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if isinstance(v, ctypes.Array):
                v = list(v)[:dim]
            out[name] = v
        return out


_lib = None


def load() -> ctypes.CDLL:
    """Load libiblb.so; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library not built: {LIB_PATH} is missing "
            "(run `python -m paper_2503_20605_amd.build` or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    c_int, c_void_p, c_size_t, c_double = ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double
    ip = P(c_int)
    lib.iblb_workspace_bytes.argtypes = [c_int, P(iblb_params), ip, ip, c_int]
    lib.iblb_workspace_bytes.restype = c_size_t
    lib.iblb_create.argtypes = [c_int, P(iblb_params), ip, ip, c_int, c_void_p, c_size_t,
                                c_void_p, P(c_void_p)]
    lib.iblb_destroy.argtypes = [c_void_p]
    lib.iblb_last_error.argtypes = [c_void_p]
    lib.iblb_last_error.restype = ctypes.c_char_p
    lib.iblb_set_interface.argtypes = [c_void_p, c_int, c_void_p, c_void_p]
    lib.iblb_init_rest.argtypes = [c_void_p, c_int]
    lib.iblb_init_fields.argtypes = [c_void_p, c_int, c_void_p, c_void_p]
    lib.iblb_write_populations.argtypes = [c_void_p, c_int, c_void_p]
    lib.iblb_read_populations.argtypes = [c_void_p, c_int, c_void_p]
    lib.iblb_set_force_field.argtypes = [c_void_p, c_int, c_void_p]
    lib.iblb_step.argtypes = [c_void_p, c_int]
    lib.iblb_read_fields.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    lib.iblb_read_nodes.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    lib.iblb_diagnostics.argtypes = [c_void_p, c_int, P(iblb_diag)]
    lib.iblb_set_lb_variant.argtypes = [c_void_p, c_int, ip]
    lib.iblb_autotune.argtypes = [c_void_p, c_int, ctypes.c_char_p, ip, P(c_double)]
    lib.iblb_probe_copy.argtypes = [c_void_p, c_void_p, c_size_t, c_int, c_void_p, P(c_double)]
    lib.iblb_run_to_rest.argtypes = [c_void_p, c_double, c_double, c_int, c_int, ctypes.c_longlong,
                                     P(ctypes.c_longlong)]
    lib.iblb_set_graph_steps.argtypes = [c_void_p, c_int]
    lib.iblb_set_active.argtypes = [c_void_p, c_int, c_int]
    lib.iblb_set_viscosity_ratio.argtypes = [c_void_p, c_int, c_double]
    lib.iblb_inside_mask.argtypes = [c_void_p, c_int, c_void_p]
    lib.iblb_contact_radius.argtypes = [c_void_p, c_int, c_double, c_double, P(c_double)]
    lib.iblb_set_membrane_shear.argtypes = [c_void_p, c_int, c_double]
    lib.iblb_set_node_respacing.argtypes = [c_void_p, c_int, c_double]
    lib.iblb_set_timing.argtypes = [c_void_p, c_int]
    lib.iblb_last_timing.argtypes = [c_void_p, P(c_double), P(c_double)]
    lib.iblb_time_lattice.argtypes = [c_void_p, c_int, P(c_double)]
    lib.iblb_mlp_workspace_bytes.argtypes = [c_int, ip, c_int]
    lib.iblb_mlp_workspace_bytes.restype = c_size_t
    lib.iblb_mlp_create.argtypes = [c_int, ip, c_int, c_void_p, c_size_t, c_void_p, P(c_void_p)]
    lib.iblb_mlp_destroy.argtypes = [c_void_p]
    lib.iblb_mlp_last_error.argtypes = [c_void_p]
    lib.iblb_mlp_last_error.restype = ctypes.c_char_p
    lib.iblb_mlp_param_count.argtypes = [c_void_p]
    lib.iblb_mlp_param_count.restype = ctypes.c_longlong
    lib.iblb_mlp_set_params.argtypes = [c_void_p, c_void_p]
    lib.iblb_mlp_get_params.argtypes = [c_void_p, c_void_p]
    lib.iblb_mlp_forward.argtypes = [c_void_p, c_void_p, c_int, c_void_p]
    lib.iblb_mlp_forward_noalloc.argtypes = [c_void_p, c_void_p, c_int, c_void_p]
    lib.iblb_mlp_gradients.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p, P(c_double)]
    lib.iblb_mlp_adam_step.argtypes = [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float]
    for name in EXPORTED:
        if name not in ("iblb_workspace_bytes", "iblb_last_error", "iblb_mlp_workspace_bytes",
                        "iblb_mlp_last_error", "iblb_mlp_param_count"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


class IblbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, ctx=None):
    if code != IBLB_OK:
        msg = load().iblb_last_error(ctx)
        raise IblbError(code, msg.decode() if msg else "")
    return code


def check_mlp(code, mlp=None):
    if code != IBLB_OK:
        msg = load().iblb_mlp_last_error(mlp)
        raise IblbError(code, msg.decode() if msg else "")
    return code
