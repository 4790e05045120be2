"""ctypes declarations of libnnp's C ABI (include/nnp.h).  Marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnp.so")

c_float_p = ctypes.POINTER(ctypes.c_float)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_void_p = ctypes.c_void_p

NNP_OK, NNP_E_ARG, NNP_E_CAPACITY, NNP_E_BOX, NNP_E_NONFINITE, NNP_E_NOMEM, NNP_E_BUSY, \
    NNP_E_PENDING, NNP_E_HIP, NNP_E_ROW, NNP_E_SCRATCH = range(11)
NNP_FP32, NNP_BF16_MLP = 0, 1
STATUS_NAMES = ["NNP_OK", "NNP_E_ARG", "NNP_E_CAPACITY", "NNP_E_BOX", "NNP_E_NONFINITE",
                "NNP_E_NOMEM", "NNP_E_BUSY", "NNP_E_PENDING", "NNP_E_HIP", "NNP_E_ROW", "NNP_E_SCRATCH"]
NNP_STATIC_SCRATCH_BYTES = 64 << 20
NNP_MAX_ROW = 256
NNP_MAX_ANGULAR = 96
STAGES = ["neighbors", "group", "aev", "mlp", "energy", "aev_adjoint", "forces", "integrate"]

# symbol -> (restype, argtypes)
SIGNATURES = {
    "nnp_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "nnp_model_create": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int, ctypes.POINTER(c_void_p)]),
    "nnp_model_destroy": (None, [c_void_p]),
    "nnp_model_set_precision": (ctypes.c_int, [c_void_p, ctypes.c_int]),
    "nnp_aev_dim": (ctypes.c_int32, [c_void_p]),
    "nnp_model_fused_mlp": (ctypes.c_int32, [c_void_p]),
    "nnp_model_set_fused_mlp": (ctypes.c_int, [c_void_p, ctypes.c_int32]),
    "nnp_check": (ctypes.c_int, [c_void_p, c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "nnp_neighbors_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, c_void_p, ctypes.c_float]),
    "nnp_neighbors": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, ctypes.c_int32, c_void_p,
                                     ctypes.c_float, c_void_p, ctypes.POINTER(ctypes.c_int64), c_void_p,
                                     ctypes.c_size_t, c_void_p]),
    "nnp_workspace_bytes": (ctypes.c_size_t, [c_void_p, ctypes.c_int32, ctypes.c_int64]),
    "nnp_energy_forces": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p, ctypes.c_int32,
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                         ctypes.c_size_t, c_void_p]),
    "nnp_energy_forces_static": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                                ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                                c_void_p]),
    "nnp_energy_forces_virial": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                                ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                                c_void_p, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "nnp_model_create_ensemble": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int32, ctypes.c_int,
                                                 ctypes.POINTER(c_void_p)]),
    "nnp_model_nets": (ctypes.c_int32, [c_void_p]),
    "nnp_energy_forces_ensemble": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p,
                                                  ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                                  c_void_p, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "nnp_aev": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, ctypes.c_size_t, c_void_p]),
    "nnp_mlp": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               ctypes.c_size_t, c_void_p]),
    "nnp_md_kick_drift": (ctypes.c_int, [ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float,
                                         c_void_p, c_void_p, c_void_p]),
    "nnp_md_kick": (ctypes.c_int, [ctypes.c_int32, c_void_p, c_void_p, c_void_p, ctypes.c_float, c_void_p]),
    "nnp_md_wrap": (ctypes.c_int, [ctypes.c_int32, c_void_p, c_void_p, c_void_p]),
    "nnp_md_create": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "nnp_md_run": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p]),
    "nnp_md_get": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nnp_md_log": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), c_void_p]),
    "nnp_md_info": (ctypes.c_int, [c_void_p, c_void_p, c_void_p]),
    "nnp_md_destroy": (None, [c_void_p]),
    "nnp_server_create": (ctypes.c_int, [c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(c_void_p)]),
    "nnp_submit": (ctypes.c_int, [c_void_p, ctypes.c_int32, c_void_p, c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "nnp_poll": (ctypes.c_int, [c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), c_void_p]),
    "nnp_server_stats": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "nnp_server_destroy": (None, [c_void_p]),
    "nnp_profile_enable": (ctypes.c_int, [c_void_p, ctypes.c_int]),
    "nnp_profile_enable_mask": (ctypes.c_int, [c_void_p, ctypes.c_uint32]),
    "nnp_profile_read": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}


class AevParams(ctypes.Structure):
    _fields_ = [
        ("n_species", ctypes.c_int32), ("rc_r", ctypes.c_float), ("eta_r", ctypes.c_float),
        ("n_shf_r", ctypes.c_int32), ("shf_r", c_float_p),
        ("rc_a", ctypes.c_float), ("eta_a", ctypes.c_float), ("zeta", ctypes.c_float),
        ("n_shf_a", ctypes.c_int32), ("n_shf_z", ctypes.c_int32),
        ("shf_a", c_float_p), ("shf_z", c_float_p),
        ("radial_prefactor", ctypes.c_float), ("cos_scale", ctypes.c_float),
    ]


class MlpParams(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32), ("widths", c_int32_p),
        ("W", ctypes.POINTER(c_float_p)), ("b", ctypes.POINTER(c_float_p)),
        ("celu_alpha", ctypes.c_float), ("self_energy", ctypes.POINTER(ctypes.c_double)),
    ]


class NList(ctypes.Structure):
    _fields_ = [
        ("row_ptr", c_void_p), ("col", c_void_p), ("shift", c_void_p), ("rev", c_void_p),
        ("capacity", ctypes.c_int64), ("r_list", ctypes.c_float), ("n_atoms", ctypes.c_int32),
        ("n_pairs", ctypes.c_int64),
    ]


class MdParams(ctypes.Structure):
    _fields_ = [
        ("integrator", ctypes.c_int32), ("dt", ctypes.c_float), ("temperature", ctypes.c_float),
        ("friction", ctypes.c_float), ("seed", ctypes.c_uint64), ("skin", ctypes.c_float),
        ("rebuild_every", ctypes.c_int32), ("trigger", ctypes.c_float), ("log_every", ctypes.c_int32),
        ("log_capacity", ctypes.c_int32),
    ]


class MdStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("rebuilds", ctypes.c_int64), ("early_rebuilds", ctypes.c_int64),
        ("capacity", ctypes.c_int64), ("r_list", ctypes.c_float),
    ]


_lib = None


class NNPError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__("%s failed: %s" % (where, name))


def lib():
    """The loaded library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnnp.so is not built; run paper_2405_01491_amd.build.build() "
                               "(hipcc, gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, where):
    if status != NNP_OK:
        raise NNPError(status, where)
