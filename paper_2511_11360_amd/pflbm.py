"""ctypes binding of libpflbm.so: the C ABI of include/pflbm.h, same names,
argument marshalling only. Loading fails loudly when the library is missing.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpflbm.so")

PFLBM_OK = 0
PFLBM_EINVAL = -1
PFLBM_EUNSUPPORTED = -2
PFLBM_EHIP = -3
PFLBM_EUNSTABLE = -4
PFLBM_ESTATE = -5

PFLBM_D2Q9_D2Q5 = 0
PFLBM_D3Q19_D3Q7 = 1
PFLBM_D3Q27_D3Q7 = 2
LATTICES = {"D2Q9_D2Q5": PFLBM_D2Q9_D2Q5, "D3Q19_D3Q7": PFLBM_D3Q19_D3Q7, "D3Q27_D3Q7": PFLBM_D3Q27_D3Q7}
PFLBM_AC = 0
PFLBM_CH = 1
PFLBM_NL = 2
PFLBM_L18 = 3
PFLBM_L14 = 4
MODELS = {"AC": PFLBM_AC, "CH": PFLBM_CH, "NL": PFLBM_NL, "L18": PFLBM_L18, "L14": PFLBM_L14}
PFLBM_FP64 = 0
PFLBM_FP32 = 1
PFLBM_MIXED_FP16 = 2
PFLBM_MIXED_BF16 = 3
PFLBM_PERIODIC = 0
PFLBM_WALL = 1
PFLBM_VISC_LINEAR_MU = 0
PFLBM_VISC_LINEAR_NU = 1
PFLBM_PROBE_CHUNKS = 0
PFLBM_PROBE_TILES = 1
PFLBM_PROBE_SHIFT_LD = 2
PFLBM_PROBE_SHIFT_ST = 3
PFLBM_PROBE_ZSKEW = 4

PRECISIONS = {"fp64": PFLBM_FP64, "fp32": PFLBM_FP32, "mixed_fp16": PFLBM_MIXED_FP16,
              "mixed_bf16": PFLBM_MIXED_BF16}


class pflbm_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("model", ctypes.c_int), ("precision", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc", ctypes.c_int * 3),
        ("wall_u", (ctypes.c_double * 3) * 2),
        ("rho_H", ctypes.c_double), ("rho_L", ctypes.c_double),
        ("nu_H", ctypes.c_double), ("nu_L", ctypes.c_double),
        ("visc_interp", ctypes.c_int),
        ("M", ctypes.c_double), ("W", ctypes.c_double), ("sigma", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("gravity", ctypes.c_double * 3), ("force", ctypes.c_double * 3),
        ("s_other", ctypes.c_double), ("normal_eps", ctypes.c_double), ("lam", ctypes.c_double),
        ("freeze_phi", ctypes.c_int), ("check_interval", ctypes.c_int), ("zblock", ctypes.c_int),
        ("tile", ctypes.c_int),
    ]


class pflbm_diag(ctypes.Structure):
    _fields_ = [
        ("V_phi", ctypes.c_double), ("V_count", ctypes.c_double), ("sum_phi", ctypes.c_double),
        ("phi_min", ctypes.c_double), ("phi_max", ctypes.c_double), ("umax", ctypes.c_double),
        ("p_in", ctypes.c_double), ("p_out", ctypes.c_double),
        ("n_in", ctypes.c_longlong), ("n_out", ctypes.c_longlong),
        ("unstable", ctypes.c_int),
    ]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "pflbm_state_bytes": (ctypes.c_int, [ctypes.POINTER(pflbm_params), ctypes.POINTER(ctypes.c_size_t)]),
    "pflbm_create": (ctypes.c_int, [ctypes.POINTER(pflbm_params), _P, _P, ctypes.c_size_t,
                                    ctypes.POINTER(_P)]),
    "pflbm_init": (ctypes.c_int, [_P, _P, _P, _P]),
    "pflbm_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "pflbm_fields": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "pflbm_volume": (ctypes.c_int, [_P, _D, ctypes.c_double, ctypes.POINTER(pflbm_diag)]),
    "pflbm_get_distributions": (ctypes.c_int, [_P, _P, _P]),
    "pflbm_set_distributions": (ctypes.c_int, [_P, _P, _P]),
    "pflbm_step_count": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_longlong)]),
    "pflbm_checkpoint_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "pflbm_save_state": (ctypes.c_int, [_P, _P]),
    "pflbm_load_state": (ctypes.c_int, [_P, _P]),
    "pflbm_adjoint_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "pflbm_adjoint_step": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pflbm_adjoint_init": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "pflbm_adjoint_seed_phi": (ctypes.c_int, [_P, _P, _P, _P]),
    "pflbm_adjoint_step_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "pflbm_adjoint_step_pu": (ctypes.c_int, [_P] * 12),
    "pflbm_adjoint_seed": (ctypes.c_int, [_P] * 7),
    "pflbm_get_distributions_f32": (ctypes.c_int, [_P] * 3),
    "pflbm_step_record": (ctypes.c_int, [_P] * 4),
    "pflbm_step_record_f32": (ctypes.c_int, [_P] * 4),
    "pflbm_adjoint_step_pu_f32": (ctypes.c_int, [_P] * 12),
    "pflbm_adjoint_init_pu_f32": (ctypes.c_int, [_P] * 10),
    "pflbm_adjoint_step_f32": (ctypes.c_int, [_P] * 9),
    "pflbm_adjoint_seed_phi_f32": (ctypes.c_int, [_P] * 4),
    "pflbm_adjoint_init_f32": (ctypes.c_int, [_P] * 7),
    "pflbm_adjoint_init_pu": (ctypes.c_int, [_P] * 10),
    "pflbm_get_phiu": (ctypes.c_int, [_P, _P]),
    "pflbm_set_phiu": (ctypes.c_int, [_P, _P]),
    "pflbm_probe_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "pflbm_probe_stream": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, _P]),
    "pflbm_destroy": (None, [_P]),
    "pflbm_last_error": (ctypes.c_char_p, [_P]),
    "pflbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def lib():
    """Load libpflbm.so (once). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpflbm.so is not built (run paper_2511_11360_amd.build); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PflbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (lib().pflbm_strerror(status).decode(), status, msg))
        self.status = status


TILES = {"auto": 0, "64x4": 1, "128x2": 2, "256x1": 3, "256x4": 4, "128x8": 5}


def make_params(d, precision="fp64", check_interval=0, zblock=0, tile="auto"):
    """pflbm_params from a workload dict (keys as in workloads.base_params)."""
    p = pflbm_params()
    p.lattice = LATTICES[d["lattice"]]
    p.model = MODELS[d["model"]]
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.nx, p.ny, p.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    for a in range(3):
        p.bc[a] = PFLBM_WALL if d["bc"][a] == "wall" else PFLBM_PERIODIC
    for s in range(2):
        for a in range(3):
            p.wall_u[s][a] = float(d["wall_u"][s][a])
    p.rho_H, p.rho_L = float(d["rho_H"]), float(d["rho_L"])
    p.nu_H, p.nu_L = float(d["nu_H"]), float(d["nu_L"])
    p.visc_interp = PFLBM_VISC_LINEAR_MU if d.get("visc_interp", "mu") == "mu" else PFLBM_VISC_LINEAR_NU
    p.M, p.W, p.sigma = float(d["M"]), float(d["W"]), float(d["sigma"])
    p.eta = float(d.get("eta", 1.0))
    for a in range(3):
        p.gravity[a] = float(d["gravity"][a])
        p.force[a] = float(d["force"][a])
    p.s_other = float(d.get("s_other", 1.0))
    p.normal_eps = float(d.get("normal_eps", 1e-4))
    p.lam = float(d.get("lam", 0.0))
    p.freeze_phi = 1 if d.get("freeze_phi", False) else 0
    p.check_interval = int(check_interval)
    p.zblock = int(zblock)
    p.tile = TILES[tile] if isinstance(tile, str) else int(tile)
    return p
