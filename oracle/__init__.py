"""FP64 CPU oracle for HMM inference (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The GPU library never does, and nothing here is
shared with it.  ``build()`` compiles ``hmm_oracle.c`` with gcc into
``liboracle.so`` next to this file; the functions below are thin ctypes
wrappers that marshal numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FAMILY_CODES = {"gaussian": 0, "gamma": 1, "student_t": 2, "poisson": 3,
                "diag": 4, "full": 5, "table": 6}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class MOpts(ctypes.Structure):
    _fields_ = [("eps_collapse", ctypes.c_double), ("ridge", ctypes.c_double),
                ("gamma_rtol", ctypes.c_double), ("nu_tol", ctypes.c_double),
                ("nu_min", ctypes.c_double), ("nu_max", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("t_nu_printed", ctypes.c_int32)]


def default_mopts(**kw) -> MOpts:
    o = MOpts(1e-8, 1e-6, 1e-12, 1e-6, 0.5, 1e4, 100, 0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oracle_lse.argtypes = [P, ctypes.c_int]
    lib.oracle_lse.restype = f64
    lib.oracle_digamma.argtypes = [f64]
    lib.oracle_digamma.restype = f64
    lib.oracle_trigamma.argtypes = [f64]
    lib.oracle_trigamma.restype = f64
    lib.oracle_emission.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, i64, P, P]
    lib.oracle_forward.argtypes = [ctypes.c_int, P, P, i64, P, P]
    lib.oracle_backward.argtypes = [ctypes.c_int, P, i64, P, P]
    lib.oracle_posteriors.argtypes = [ctypes.c_int, P, i64, P, P, P, f64, P, P, P]
    lib.oracle_stats_len.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_stats_len.restype = i64
    lib.oracle_estep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, i64, P, P,
                                 P, P, P, P, P, P]
    lib.oracle_viterbi.argtypes = [ctypes.c_int, P, P, i64, P, f64, P, P, P]
    lib.oracle_posterior_decode.argtypes = [ctypes.c_int, i64, P, P]
    lib.oracle_mstep_transitions.argtypes = [ctypes.c_int, P, P, f64, P, P, P]
    lib.oracle_mstep_emission.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P,
                                          ctypes.POINTER(MOpts), P, P, P]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lse(x) -> float:
    x = _f64(x)
    return _load().oracle_lse(_p(x), x.size)


def digamma(x: float) -> float:
    return _load().oracle_digamma(float(x))


def trigamma(x: float) -> float:
    return _load().oracle_trigamma(float(x))


def emission(family: str, n: int, d: int, theta, obs) -> np.ndarray:
    """log b_j(y_t) as [T, N]."""
    obs = _f64(obs).reshape(-1, d)
    theta = _f64(theta)
    T = obs.shape[0]
    out = np.empty((T, n), dtype=np.float64)
    _load().oracle_emission(FAMILY_CODES[family], n, d, _p(theta), T, _p(obs), _p(out))
    return out


def forward(log_pi, log_A, logB) -> np.ndarray:
    log_pi, log_A, logB = _f64(log_pi), _f64(log_A), _f64(logB)
    T, n = logB.shape
    out = np.empty((T, n))
    _load().oracle_forward(n, _p(log_pi), _p(log_A), T, _p(logB), _p(out))
    return out


def backward(log_A, logB) -> np.ndarray:
    log_A, logB = _f64(log_A), _f64(logB)
    T, n = logB.shape
    out = np.empty((T, n))
    _load().oracle_backward(n, _p(log_A), T, _p(logB), _p(out))
    return out


def posteriors(log_A, logB, alpha, beta, loglik, want_xi=True):
    """Returns (gamma [T,N], xi [T-1,N,N] or None, xi_sum [N,N])."""
    log_A, logB, alpha, beta = _f64(log_A), _f64(logB), _f64(alpha), _f64(beta)
    T, n = logB.shape
    gamma = np.empty((T, n))
    xi = np.empty((max(T - 1, 0), n, n)) if want_xi else None
    xs = np.empty((n, n))
    _load().oracle_posteriors(n, _p(log_A), T, _p(logB), _p(alpha), _p(beta), float(loglik),
                              _p(gamma), _p(xi), _p(xs))
    return gamma, xi, xs


def stats_len(family: str, n: int, d: int = 1) -> int:
    return int(_load().oracle_stats_len(FAMILY_CODES[family], n, d))


def estep(model, offsets, obs, logB=None, want_gamma=False):
    """Pooled E-step over a ragged batch.

    Returns dict(stats, loglik, loglik_bwd, status, gamma)."""
    fam = model.family
    n, d = model.n_states, model.dim
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    B = len(offsets) - 1
    obs_a = None if obs is None else _f64(obs).reshape(-1, d)
    logB_a = None if logB is None else _f64(logB)
    stats = np.empty(stats_len(fam, n, d))
    ll = np.empty(B)
    ll2 = np.empty(B)
    st = np.empty(B, dtype=np.int32)
    gam = np.empty((int(offsets[-1]), n)) if want_gamma else None
    rc = _load().oracle_estep(FAMILY_CODES[fam], n, d, _p(_f64(model.log_pi)),
                              _p(_f64(model.log_A)), _p(_f64(model.theta)), B, _p(offsets),
                              _p(obs_a), _p(logB_a), _p(stats), _p(ll), _p(ll2), _p(st), _p(gam))
    if rc != 0:
        raise ValueError("oracle_estep: bad arguments")
    return {"stats": stats, "loglik": ll, "loglik_bwd": ll2, "status": st, "gamma": gam}


def viterbi(log_pi, log_A, logB, tie_eps=1e-12):
    """Returns (path [T] int32, logp, n_ties)."""
    log_pi, log_A, logB = _f64(log_pi), _f64(log_A), _f64(logB)
    T, n = logB.shape
    path = np.empty(T, dtype=np.int32)
    lp = ctypes.c_double()
    nt = ctypes.c_int32()
    _load().oracle_viterbi(n, _p(log_pi), _p(log_A), T, _p(logB), float(tie_eps), _p(path),
                           ctypes.byref(lp), ctypes.byref(nt))
    return path, lp.value, nt.value


def posterior_decode(gamma) -> np.ndarray:
    gamma = _f64(gamma)
    T, n = gamma.shape
    path = np.empty(T, dtype=np.int32)
    _load().oracle_posterior_decode(n, T, _p(gamma), _p(path))
    return path


def mstep_transitions(n, stats, log_A_old, eps=1e-8):
    stats, log_A_old = _f64(stats), _f64(log_A_old)
    lp = np.empty(n)
    la = np.empty((n, n))
    kept = np.empty(n, dtype=np.int32)
    _load().oracle_mstep_transitions(n, _p(stats), _p(log_A_old), float(eps), _p(lp), _p(la),
                                     _p(kept))
    return lp, la, kept


def mstep_emission(family, n, d, theta_old, stats, opts: Optional[MOpts] = None):
    """Returns (theta_new, collapsed [N], iters [N])."""
    theta_old, stats = _f64(theta_old), _f64(stats)
    opts = opts if opts is not None else default_mopts()
    out = np.empty_like(theta_old)
    col = np.zeros(n, dtype=np.int32)
    it = np.zeros(n, dtype=np.int32)
    rc = _load().oracle_mstep_emission(FAMILY_CODES[family], n, d, _p(theta_old), _p(stats),
                                       ctypes.byref(opts), _p(out), _p(col), _p(it))
    if rc != 0:
        raise ValueError("unsupported family for the M-step")
    return out, col, it


def em_iteration(model, offsets, obs, opts: Optional[MOpts] = None):
    """One Baum-Welch iteration (E-step then M-step); returns (new_model, estep_result)."""
    r = estep(model, offsets, obs)
    n, d = model.n_states, model.dim
    lp, la, _ = mstep_transitions(n, r["stats"], model.log_A,
                                  (opts or default_mopts()).eps_collapse)
    th, _, _ = mstep_emission(model.family, n, d, model.theta, r["stats"], opts)
    m = model.copy()
    m.log_pi, m.log_A, m.theta = lp, la, th
    return m, r
