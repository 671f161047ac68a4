"""ctypes binding of libscola.so: argument marshalling only.

Every numerical step runs in the HIP library; this module converts Python/torch arguments
to the C ABI of include/scola.h and raises on any non-zero status.  It never falls back
to another implementation: if the library is missing, loading fails loudly.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscola.so")

SCOLA_FP32, SCOLA_FP64 = 0, 1
SCOLA_BATCHED, SCOLA_PER_TILE = 0, 1
SCOLA_MODIFIED, SCOLA_STANDARD = 0, 1
FIXED_BITS = 40
STATIC_WORKSPACE_BYTES = 128 << 20   # SCOLA_STATIC_WORKSPACE_BYTES

STATUS = {0: "SCOLA_OK", -1: "SCOLA_EINVAL", -2: "SCOLA_ENOMEM", -3: "SCOLA_EDEVICE",
          -4: "SCOLA_ESTATE", -5: "SCOLA_EUNSUPPORTED", -6: "SCOLA_EOVERFLOW"}


class ScolaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Cosmology(ctypes.Structure):
    _fields_ = [("Omega_m", ctypes.c_double), ("Omega_b", ctypes.c_double),
                ("h", ctypes.c_double), ("n_s", ctypes.c_double),
                ("sigma8", ctypes.c_double), ("T_cmb", ctypes.c_double)]


class Tile(ctypes.Structure):
    _fields_ = [("core_lo", ctypes.c_int32 * 3), ("core_n", ctypes.c_int32),
                ("buffer", ctypes.c_int32), ("mesh", ctypes.c_int32 * 3),
                ("a_f", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("Np", ctypes.c_int32), ("N_lpt", ctypes.c_int32),
                ("N_out", ctypes.c_int32), ("fda_order", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("a_i", ctypes.c_double),
                ("a_f", ctypes.c_double), ("n_lpt", ctypes.c_double),
                ("discretisation", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("want_momenta", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32)]


def make_config(L, Np, n_steps, a_i, a_f, precision, schedule, want_momenta=0, N_out=0,
                checkpoint_every=0, N_lpt=0, fda_order=0, n_lpt=0.0, discretisation=0):
    """A Config with the fields named as in include/scola.h (zero = the default)."""
    return Config(L=float(L), Np=int(Np), N_lpt=int(N_lpt), N_out=int(N_out),
                  fda_order=int(fda_order), n_steps=int(n_steps), a_i=float(a_i),
                  a_f=float(a_f), n_lpt=float(n_lpt), discretisation=int(discretisation),
                  precision=int(precision), schedule=int(schedule),
                  want_momenta=int(want_momenta), checkpoint_every=int(checkpoint_every))


class Layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_size_t) for n in
                ("psi1", "psi2", "x_res", "p_res", "rho", "work", "phi", "bc0", "dropped",
                 "cells", "phi1", "phi2", "cbuf", "outgrid", "ckpt", "seg_x", "seg_phi", "lam_x",
                 "lam_p", "lam_psi1", "lam_psi2", "lam_rho", "lam_bc0", "adj_grid",
                 "total")] + \
               [("n_particles", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_padded", ctypes.c_int64), ("fixed_bits", ctypes.c_int32)]


class ClassSchedule(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("xcd_remap_particles", ctypes.c_int32), ("xcd_remap_mesh", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32
_SIGS = {
    "scola_status_string": ([_I], ctypes.c_char_p),
    "scola_last_error": ([], ctypes.c_char_p),
    "scola_uniform_tiling": ([_I, _I, _I, ctypes.POINTER(Tile), _I], _I),
    "scola_plan_create": ([ctypes.POINTER(Config), ctypes.POINTER(Cosmology),
                           ctypes.POINTER(Tile), _I, ctypes.POINTER(_P)], _I),
    "scola_plan_destroy": ([_P], _I),
    "scola_workspace_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I),
    "scola_workspace_layout": ([_P, ctypes.POINTER(Layout)], _I),
    "scola_forward": ([_P, _P, _P, _P, _P, ctypes.POINTER(_I), _I, _P, _P], _I),
    "scola_forward_noalloc": ([_P, _P, _P, _P, _P, _P], _I),
    "scola_setup": ([_P, _P, _P, _P], _I),
    "scola_backward": ([_P, _P, _P, _P, _P], _I),
    "scola_evolve": ([_P, ctypes.POINTER(_I), _I, _P, _P], _I),
    "scola_output": ([_P, _P, _P, _P, ctypes.POINTER(_I), _I, _P, _P], _I),
    "scola_op_deposit": ([_P, _D, _D, _P, _P], _I),
    "scola_op_poisson": ([_P, _D, _P, _P], _I),
    "scola_op_step": ([_P, _D, _D, _D, _D, _D, _D, _I, _P, _P], _I),
    "scola_op_final_kick": ([_P, _D, _D, _D, _D, _D, _P, _P], _I),
    "scola_step_table": ([_P, ctypes.POINTER(_D), _I], _I),
    "scola_power_spectrum": ([_P, ctypes.POINTER(_D), ctypes.POINTER(_D), _I], _I),
    "scola_schedule_table": ([ctypes.POINTER(Config), ctypes.POINTER(Cosmology),
                              ctypes.POINTER(_D), _I], _I),
    "scola_linear_power": ([ctypes.POINTER(Cosmology), ctypes.POINTER(_D), ctypes.POINTER(_D),
                            _I], _I),
    "scola_plan_tune": ([_P, _P, _P, _I], _I),
    "scola_plan_set_graph": ([_P, _I], _I),
    "scola_plan_set_persistent": ([_P, _I], _I),
    "scola_plan_persistent": ([_P, _P, ctypes.POINTER(_I), ctypes.POINTER(_I),
                               ctypes.POINTER(_I)], _I),
    "scola_plan_concurrency": ([_P, ctypes.POINTER(_I)], _I),
    "scola_plan_set_concurrency": ([_P, _I], _I),
    "scola_plan_schedule": ([_P, _P, _I, ctypes.POINTER(_I)], _I),
    "scola_plan_set_schedule": ([_P, _P, _I], _I),
    "scola_evolve_overrides": ([_P, _P, _P, _P, _P], _I),
    "scola_tcola_workspace_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I),
    "scola_tcola_forward": ([_P, _P, _P, _P, _P, _P, _P, _P, _P], _I),
    "scola_mass_alarm": ([_P, _P, _P, ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64)], _I),
    "scola_plan_info": ([_P, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_int64),
                         ctypes.POINTER(_D), ctypes.POINTER(_D)], _I),
}


def lib():
    """Load libscola.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2003_04925_amd.build` (no fallback exists)")
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def check(status):
    if status != 0:
        msg = lib().scola_last_error().decode(errors="replace")
        raise ScolaError(status, msg)


def exported_symbols():
    return sorted(_SIGS)
