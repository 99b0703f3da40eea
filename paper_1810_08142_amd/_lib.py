"""ctypes binding of ``libriccsd.so`` (argument marshalling only).

The library must have been built (``python -m paper_1810_08142_amd.build`` or
``__graft_entry__.build()``); there is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libriccsd.so")

_c = ctypes
_dp = _c.c_void_p  # device pointers travel as plain addresses
_lib = None


class RIError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class RISystem(_c.Structure):
    _fields_ = [("o", _c.c_int), ("v", _c.c_int), ("naux", _c.c_int), ("B", _dp), ("eps", _dp)]


class RICcsdOpts(_c.Structure):
    _fields_ = [("max_iter", _c.c_int), ("tol_residual", _c.c_double), ("tol_energy", _c.c_double),
                ("diis_size", _c.c_int), ("diis_start", _c.c_int), ("ppl_precision", _c.c_int),
                ("guess", _c.c_int), ("verbose", _c.c_int), ("polish_residual", _c.c_double),
                ("check_fp64", _c.c_int), ("mlp", _c.c_void_p), ("polish_precision", _c.c_int),
                ("other_precision", _c.c_int)]


class RICcsdReport(_c.Structure):
    _fields_ = [("e_corr", _c.c_double), ("e_mp2", _c.c_double), ("residual_inf", _c.c_double),
                ("iterations", _c.c_int), ("converged", _c.c_int), ("seconds_total", _c.c_double),
                ("seconds_ppl", _c.c_double), ("residual_rms", _c.c_double), ("residual_inf_fp64", _c.c_double),
                ("polish_iteration", _c.c_int), ("seconds_guess", _c.c_double), ("guess_used", _c.c_int)]


class RIMlpTrainOpts(_c.Structure):
    _fields_ = [("epochs", _c.c_int), ("batch", _c.c_long), ("lr", _c.c_float), ("warmup", _c.c_float),
                ("seed", _c.c_ulonglong), ("shuffle", _c.c_int)]


_sysp = _c.POINTER(RISystem)
_dblp = _c.POINTER(_c.c_double)
_fltp = _c.POINTER(_c.c_float)

# (name, restype, argtypes)
_SIGS = [
    ("ri_status_str", _c.c_char_p, [_c.c_int]),
    ("ri_last_error_msg", _c.c_char_p, []),
    ("ri_last_hip_error", _c.c_int, []),
    ("ri_ppl", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _dp]),
    ("ri_ppl_ex", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _c.c_int, _dp, _c.c_size_t, _dp]),
    ("ri_ppl_shard", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _c.c_int, _c.c_int, _c.c_int, _dp,
                                _c.c_size_t, _dp]),
    ("ri_ppl_paper", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _dp]),
    ("ri_ppl_paper_flops", _c.c_double, [_c.c_int, _c.c_int, _c.c_int]),
    ("ri_ppl_sym", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _dp]),
    ("ri_ppl_sym_ex", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _c.c_int, _dp]),
    ("ri_ppl_noalloc", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _c.c_int, _dp, _c.c_int, _dp]),
    ("ri_ppl_sym_flops", _c.c_double, [_c.c_int, _c.c_int, _c.c_int]),
    ("ri_ppl_workspace_bytes", _c.c_size_t, [_c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    ("ri_ppl_flops", _c.c_double, [_c.c_int, _c.c_int, _c.c_int]),
    ("ri_build_tau", _c.c_int, [_dp, _dp, _c.c_int, _c.c_int, _dp, _dp]),
    ("ri_tau_pair_asymmetry", _c.c_int, [_dp, _c.c_int, _c.c_int, _dblp, _dp]),
    ("ri_prof_enable", _c.c_int, [_c.c_int]),
    ("ri_prof_report", _c.c_int, [_c.c_char_p, _c.c_size_t]),
    ("ri_ccsd_default_opts", None, [_c.POINTER(RICcsdOpts)]),
    ("ri_mp2_guess", _c.c_int, [_sysp, _dp, _dp, _dblp, _dp]),
    ("ri_ccsd_energy", _c.c_int, [_sysp, _dp, _dp, _dblp, _dp]),
    ("ri_ccsd_residual", _c.c_int, [_sysp, _dp, _dp, _dp, _dp, _c.c_int, _dp]),
    ("ri_ccsd_iterate", _c.c_int, [_sysp, _dp, _dp, _c.POINTER(RICcsdOpts), _c.POINTER(RICcsdReport), _dp]),
    ("ri_ccsd_triples", _c.c_int, [_sysp, _dp, _dp, _dblp, _dp]),
    ("ri_ccsd_triples_ex", _c.c_int, [_sysp, _dp, _dp, _c.c_int, _dblp, _dp]),
    ("ri_ccsd_triples_flops", _c.c_double, [_c.c_int, _c.c_int]),
    ("ri_mlp_create", _c.c_void_p, [_c.c_int, _c.c_int, _c.c_int]),
    ("ri_mlp_destroy", None, [_c.c_void_p]),
    ("ri_mlp_num_params", _c.c_size_t, [_c.c_void_p]),
    ("ri_mlp_set_params", _c.c_int, [_c.c_void_p, _fltp]),
    ("ri_mlp_get_params", _c.c_int, [_c.c_void_p, _fltp]),
    ("ri_mlp_set_scaling", _c.c_int, [_c.c_void_p, _fltp, _fltp, _c.c_float]),
    ("ri_mlp_get_scaling", _c.c_int, [_c.c_void_p, _fltp, _fltp, _fltp]),
    ("ri_mlp_forward", _c.c_int, [_c.c_void_p, _dp, _c.c_long, _dp, _dp]),
    ("ri_mlp_infer", _c.c_int, [_c.c_void_p, _dp, _c.c_long, _dp, _dp]),
    ("ri_mlp_gradient", _c.c_int, [_c.c_void_p, _dp, _dp, _c.c_long, _dp, _fltp, _dp]),
    ("ri_mlp_train_step", _c.c_int, [_c.c_void_p, _dp, _dp, _c.c_long, _c.c_float, _fltp, _dp]),
    ("ri_mlp_init", _c.c_int, [_c.c_void_p, _c.c_ulonglong, _dp]),
    ("ri_mlp_default_train_opts", None, [_c.POINTER(RIMlpTrainOpts)]),
    ("ri_mlp_train", _c.c_int, [_c.c_void_p, _dp, _dp, _c.c_long, _dp, _dp, _c.c_long, _c.POINTER(RIMlpTrainOpts),
                                _fltp, _fltp, _dp]),
    ("ri_mlp_features", _c.c_int, [_sysp, _dp, _dp, _dp]),
    ("ri_mlp_guess", _c.c_int, [_c.c_void_p, _sysp, _dp, _dp, _dp]),
    ("ri_mlp_sample", _c.c_int, [_dp, _c.c_long, _c.c_long, _c.c_ulonglong, _dp, _dp]),
    ("ri_mlp_targets", _c.c_int, [_dp, _dp, _dp, _c.c_long, _c.c_float, _dp, _dp]),
    ("ri_mlp_fit_scaling", _c.c_int, [_c.c_void_p, _dp, _dp, _c.c_long, _dp]),
    ("ri_mlp_standardize", _c.c_int, [_c.c_void_p, _dp, _dp, _c.c_long, _dp, _dp, _dp]),
    ("ri_mlp_save", _c.c_int, [_c.c_void_p, _c.c_char_p]),
    ("ri_mlp_load", _c.c_void_p, [_c.c_char_p]),
]


def lib():
    """Load the HIP library (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_1810_08142_amd.build`)")
        L = _c.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return [s[0] for s in _SIGS]


def check(status: int, where: str):
    if status != 0:
        L = lib()
        raise RIError(status, where, L.ri_last_error_msg().decode() or L.ri_status_str(status).decode())


def prof_enable(on: bool = True):
    lib().ri_prof_enable(1 if on else 0)


def prof_report() -> list:
    """Per-kernel event timings recorded since the last report (synchronises)."""
    import json
    buf = _c.create_string_buffer(1 << 16)
    check(lib().ri_prof_report(buf, len(buf)), "ri_prof_report")
    return json.loads(buf.value.decode())
