"""ctypes declarations of libsibfa_pol.so (include/sibfa_pol.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsibfa_pol.so")

SIBFA_OK = 0
STATUS_NAMES = {0: "SIBFA_OK", -1: "SIBFA_E_ARG", -2: "SIBFA_E_STATE", -3: "SIBFA_E_NOMEM",
                -4: "SIBFA_E_NOT_SPD", -5: "SIBFA_E_NOT_CONVERGED", -6: "SIBFA_E_DEVICE"}
FP64, MIXED = 0, 1
PRECOND_DIAG, PRECOND_MOLBLOCK = 0, 1


class Params(ctypes.Structure):
    _fields_ = [("ewald_beta", ctypes.c_double), ("cutoff", ctypes.c_double),
                ("grid", ctypes.c_int * 3), ("order", ctypes.c_int),
                ("thole_a", ctypes.c_double), ("tol_debye", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("precond", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("true_rms_debye", ctypes.c_double), ("e_pol", ctypes.c_double),
                ("e_pol_variational", ctypes.c_double), ("e_elec", ctypes.c_double),
                ("e_elec_real", ctypes.c_double), ("e_elec_recip", ctypes.c_double),
                ("e_elec_self", ctypes.c_double), ("n_sites", ctypes.c_int),
                ("n_polarizable", ctypes.c_int), ("max_neighbors", ctypes.c_int)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 16), ("calls", ctypes.c_int * 16),
                ("pairs", ctypes.c_longlong * 4)]


PHASES = ["lists", "field_real", "field_recip", "spread", "fft", "matvec", "update",
          "force_real", "force_recip", "paircoef", "matvec_recip", "matvec_fp64"]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

class MdStats(ctypes.Structure):
    _fields_ = [("e_pol", ctypes.c_double), ("e_elec", ctypes.c_double),
                ("e_bond", ctypes.c_double), ("e_rep", ctypes.c_double),
                ("e_kin", ctypes.c_double),
                ("iterations", ctypes.c_int)]


class CtParams(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("cs", ctypes.c_double), ("cp", ctypes.c_double),
                ("t", ctypes.c_double), ("m", ctypes.c_double)]


# (name, restype, argtypes)
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
SIGNATURES = [
    ("sibfa_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ALLOC_FN, FREE_FN, _P]),
    ("sibfa_destroy", None, [_P]),
    ("sibfa_last_error", ctypes.c_char_p, [_P]),
    ("sibfa_default_params", None, [ctypes.POINTER(Params)]),
    ("sibfa_footprint_bytes", ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, _D,
                                                ctypes.POINTER(Params)]),
    ("sibfa_set_system", ctypes.c_int, [_P, ctypes.c_int, _P, _P, _D, ctypes.POINTER(Params)]),
    ("sibfa_update_positions", ctypes.c_int, [_P, _P]),
    ("sibfa_set_multipoles", ctypes.c_int, [_P, _P, _P, _P]),
    ("sibfa_set_polarizabilities", ctypes.c_int, [_P, _P, _P]),
    ("sibfa_set_local_frames", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("sibfa_set_predictor", ctypes.c_int, [_P, ctypes.c_int]),
    ("sibfa_tcg_energy_forces", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                               _P, _P, _P, _P]),
    ("sibfa_set_charge_transfer", ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P, _P,
                                                 _P, _P]),
    ("sibfa_ct_energy_forces", ctypes.c_int, [_P, _P, _P]),
    ("sibfa_md_init", ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P, _P, _P, ctypes.c_double,
                                     _P]),
    ("sibfa_md_run", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _P]),
    ("sibfa_md_get_state", ctypes.c_int, [_P, _P, _P]),
    ("sibfa_permanent_field", ctypes.c_int, [_P, _P]),
    ("sibfa_apply_T", ctypes.c_int, [_P, _P, _P]),
    ("sibfa_solve_induced", ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_int), _D]),
    ("sibfa_solve_tcg", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_int, _P, _D]),
    ("sibfa_energy_forces", ctypes.c_int, [_P, _D, _D, _P, _P]),
    ("sibfa_get_dipoles", ctypes.c_int, [_P, _P]),
    ("sibfa_set_dipoles", ctypes.c_int, [_P, _P]),
    ("sibfa_neighbor_counts", ctypes.c_int, [_P, _P]),
    ("sibfa_get_stats", ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    ("sibfa_set_profiling", ctypes.c_int, [_P, ctypes.c_int]),
    ("sibfa_set_profiling_phases", ctypes.c_int, [_P, ctypes.c_uint]),
    ("sibfa_get_profile", ctypes.c_int, [_P, ctypes.POINTER(Profile)]),
    ("sibfa_batch_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ALLOC_FN, FREE_FN,
                                          _P]),
    ("sibfa_batch_destroy", None, [_P]),
    ("sibfa_batch_last_error", ctypes.c_char_p, [_P]),
    ("sibfa_batch_clusters", ctypes.c_int, [_P, ctypes.c_int, _P, _P] + [_P] * 7 +
     [ctypes.POINTER(Params)] + [_P] * 7),
    ("sibfa_batch_clusters_noalloc", ctypes.c_int,
     [ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, _P, _P] + [_P] * 7 +
     [ctypes.POINTER(Params)] + [_P] * 7),
]

BATCH_MAX_SITES = 1024
BATCH_MAX_POLARIZABLE = 640
BATCH_NOALLOC_MAX_SITES = 32768
BATCH_NOALLOC_MAX_CLUSTERS = 4096

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2201_00804_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_names():
    return [name for name, _, _ in SIGNATURES]
