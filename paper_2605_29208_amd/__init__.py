"""Python binding of libhmmgpu (MI355X / gfx950 HMM inference).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libhmmgpu.so.  PyTorch supplies device memory and the stream.
The raw functions carry the C names (hmm_estep_stats, ...); the small
helpers below them allocate outputs and workspace and call the raw ones.

Importing this module requires the built library; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmmgpu.so")

# enums of include/hmm_gpu.h
HMM_OK, HMM_ERR_ARG, HMM_ERR_UNSUPPORTED, HMM_ERR_WORKSPACE, HMM_ERR_DEVICE, \
    HMM_ERR_PARAMS_UNSET, HMM_ERR_NUMERIC = range(7)
FAMILY = {"gaussian": 0, "gamma": 1, "student_t": 2, "poisson": 3, "diag": 4, "full": 5,
          "table": 6}
PREC = {"f64": 0, "f32": 1, "bf16_scaled": 2, "f16_scaled": 3, "plain_f32": 4, "plain_f64": 5}
OP = {"emission": 0, "forward_backward": 1, "estep": 2, "viterbi": 3, "posterior_decode": 4}

EXPORTED = [
    "hmm_version", "hmm_last_error", "hmm_stats_len", "hmm_workspace_size",
    "hmm_emission_logpdf", "hmm_forward_backward", "hmm_estep_stats", "hmm_estep_stats_noalloc",
    "hmm_viterbi",
    "hmm_posterior_decode", "hmm_mstep_default_opts", "hmm_mstep_transitions",
    "hmm_mstep_gaussian", "hmm_mstep_gamma", "hmm_mstep_student_t", "hmm_mstep_poisson",
    "hmm_mstep_diag_gaussian", "hmm_mstep_full_gaussian", "hmm_set_chunk_len",
    "hmm_profile_enable", "hmm_profile_count", "hmm_profile_get", "hmm_profile_reset",
    "hmm_autotune", "hmm_set_variant", "hmm_get_variant",
    # include/hmm_serve.h
    "hmm_server_default_opts", "hmm_server_now", "hmm_server_create", "hmm_server_destroy",
    "hmm_server_add_model", "hmm_server_submit", "hmm_server_poll", "hmm_server_get_info",
]
REQ = {"viterbi": 0, "posterior_decode": 1}


class HmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hmm status {status}: {msg}")
        self.status = status


class HmmModelC(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("family", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("log_pi", ctypes.c_void_p), ("log_A", ctypes.c_void_p),
                ("theta", ctypes.c_void_p)]


class HmmBatchC(ctypes.Structure):
    _fields_ = [("n_seq", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("h_offsets", ctypes.c_void_p), ("obs", ctypes.c_void_p),
                ("obs_f64", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class HmmMstepOptsC(ctypes.Structure):
    _fields_ = [("eps_collapse", ctypes.c_double), ("ridge", ctypes.c_double),
                ("gamma_rtol", ctypes.c_double), ("nu_tol", ctypes.c_double),
                ("nu_min", ctypes.c_double), ("nu_max", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("t_nu_printed", ctypes.c_int32)]


class HmmServerOptsC(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("host_staging", ctypes.c_size_t),
                ("max_batch", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("device", ctypes.c_int32)]


class HmmCompletionC(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("model", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("T", ctypes.c_int64), ("logp", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class HmmServerInfoC(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("in_flight", ctypes.c_int64), ("pool_bytes", ctypes.c_size_t),
                ("pool_used", ctypes.c_size_t), ("pool_peak", ctypes.c_size_t)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2605_29208_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    MP, BP = ctypes.POINTER(HmmModelC), ctypes.POINTER(HmmBatchC)
    OPP = ctypes.POINTER(HmmMstepOptsC)
    sig = {
        "hmm_version": ([], ctypes.c_char_p),
        "hmm_last_error": ([], ctypes.c_char_p),
        "hmm_stats_len": ([MP], sz),
        "hmm_workspace_size": ([ctypes.c_int, MP, BP, ctypes.c_int, ctypes.POINTER(sz)], ctypes.c_int),
        "hmm_emission_logpdf": ([MP, BP, ctypes.c_int, P, P, sz, P], ctypes.c_int),
        "hmm_forward_backward": ([MP, BP, ctypes.c_int, P, P, P, P, sz, P], ctypes.c_int),
        "hmm_estep_stats": ([MP, BP, ctypes.c_int, P, P, P, P, sz, P], ctypes.c_int),
        "hmm_estep_stats_noalloc": ([MP, BP, ctypes.c_int, P, P, P, P], ctypes.c_int),
        "hmm_viterbi": ([MP, BP, ctypes.c_int, P, P, P, P, sz, P], ctypes.c_int),
        "hmm_posterior_decode": ([MP, BP, ctypes.c_int, P, P, P, sz, P], ctypes.c_int),
        "hmm_mstep_default_opts": ([OPP], None),
        "hmm_mstep_transitions": ([MP, P, OPP, P, P, P], ctypes.c_int),
        "hmm_set_chunk_len": ([i32], ctypes.c_int),
        "hmm_autotune": ([MP, BP, ctypes.c_int, P, P, P, P, sz, P, ctypes.POINTER(i32),
                          ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "hmm_set_variant": ([i32], ctypes.c_int),
        "hmm_get_variant": ([MP, BP, ctypes.c_int, ctypes.POINTER(i32), ctypes.POINTER(i32)],
                            ctypes.c_int),
        "hmm_profile_enable": ([i32], ctypes.c_int),
        "hmm_profile_count": ([], i32),
        "hmm_profile_get": ([i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float)],
                            ctypes.c_int),
        "hmm_profile_reset": ([], ctypes.c_int),
        "hmm_server_default_opts": ([ctypes.POINTER(HmmServerOptsC)], None),
        "hmm_server_now": ([], ctypes.c_double),
        "hmm_server_create": ([ctypes.POINTER(HmmServerOptsC), ctypes.POINTER(P)], ctypes.c_int),
        "hmm_server_destroy": ([P], ctypes.c_int),
        "hmm_server_add_model": ([P, MP, ctypes.POINTER(i32)], ctypes.c_int),
        "hmm_server_submit": ([P, i32, i32, P, i32, i64, P, ctypes.POINTER(ctypes.c_uint64)],
                              ctypes.c_int),
        "hmm_server_poll": ([P, ctypes.POINTER(HmmCompletionC), i32, i32, ctypes.POINTER(i32)],
                            ctypes.c_int),
        "hmm_server_get_info": ([P, ctypes.POINTER(HmmServerInfoC)], ctypes.c_int),
    }
    for fam in ("gaussian", "gamma", "student_t", "poisson", "diag_gaussian", "full_gaussian"):
        sig[f"hmm_mstep_{fam}"] = ([MP, P, OPP, P, P, P, P], ctypes.c_int)
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def version() -> str:
    return _lib.hmm_version().decode()


def last_error() -> str:
    return _lib.hmm_last_error().decode()


def _check(st):
    if st != HMM_OK:
        raise HmmError(st, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------
# device-resident model and batch
# --------------------------------------------------------------------------

class DeviceModel:
    """lambda = (log pi, log A, theta) as FP64 device tensors."""

    def __init__(self, family, n_states, dim, log_pi, log_A, theta, device="cuda"):
        import torch
        self.family, self.n_states, self.dim = family, int(n_states), int(dim)
        f64 = dict(dtype=torch.float64, device=device)
        self.log_pi = torch.as_tensor(np.asarray(log_pi, dtype=np.float64)).to(**f64).contiguous()
        self.log_A = torch.as_tensor(np.asarray(log_A, dtype=np.float64)).to(**f64).contiguous()
        self.theta = None if theta is None else \
            torch.as_tensor(np.asarray(theta, dtype=np.float64)).to(**f64).contiguous()
        self.c = HmmModelC(self.n_states, self.dim, FAMILY[family], 0,
                           self.log_pi.data_ptr(), self.log_A.data_ptr(),
                           None if self.theta is None else self.theta.data_ptr())

    @classmethod
    def from_model(cls, m, device="cuda"):
        return cls(m.family, m.n_states, m.dim, m.log_pi, m.log_A, m.theta, device)

    def refresh(self):
        self.c.log_pi = self.log_pi.data_ptr()
        self.c.log_A = self.log_A.data_ptr()
        self.c.theta = None if self.theta is None else self.theta.data_ptr()


class DeviceBatch:
    """A ragged batch: observations [sum T, D] (float32 or float64) and offsets."""

    def __init__(self, obs, offsets, device="cuda", dtype=np.float32):
        import torch
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.h_offsets = offsets
        self.offsets = torch.as_tensor(offsets).to(device)
        obs = np.ascontiguousarray(obs, dtype=dtype)
        self.obs = torch.as_tensor(obs).to(device).contiguous()
        self.n_seq = len(offsets) - 1
        self.total = int(offsets[-1])
        self.c = HmmBatchC(self.n_seq, self.offsets.data_ptr(),
                           self.h_offsets.ctypes.data_as(ctypes.c_void_p).value,
                           self.obs.data_ptr(), 1 if dtype == np.float64 else 0, 0)

    @classmethod
    def from_workload(cls, w, dtype=np.float32, device="cuda"):
        return cls(w.obs, w.offsets, device, dtype)


# --------------------------------------------------------------------------
# raw C calls (same names as the C ABI)
# --------------------------------------------------------------------------

def hmm_stats_len(model: DeviceModel) -> int:
    return int(_lib.hmm_stats_len(ctypes.byref(model.c)))


def hmm_workspace_size(op, model: DeviceModel, batch: DeviceBatch, prec) -> int:
    out = ctypes.c_size_t()
    _check(_lib.hmm_workspace_size(OP[op], ctypes.byref(model.c), ctypes.byref(batch.c),
                                   PREC[prec], ctypes.byref(out)))
    return out.value


def hmm_emission_logpdf(model, batch, prec, log_b, ws, stream=None):
    _check(_lib.hmm_emission_logpdf(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                                    _ptr(log_b), _ptr(ws), _nbytes(ws), _stream(stream)))


def hmm_forward_backward(model, batch, prec, loglik, gamma, seq_status, ws, stream=None):
    _check(_lib.hmm_forward_backward(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                                     _ptr(loglik), _ptr(gamma), _ptr(seq_status), _ptr(ws),
                                     _nbytes(ws), _stream(stream)))


def hmm_estep_stats(model, batch, prec, stats, loglik, seq_status, ws, stream=None):
    _check(_lib.hmm_estep_stats(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                                _ptr(stats), _ptr(loglik), _ptr(seq_status), _ptr(ws),
                                _nbytes(ws), _stream(stream)))


def hmm_estep_stats_noalloc(model, batch, prec, stats, loglik, seq_status, stream=None):
    _check(_lib.hmm_estep_stats_noalloc(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                                        _ptr(stats), _ptr(loglik), _ptr(seq_status),
                                        _stream(stream)))


def hmm_viterbi(model, batch, prec, path, path_logp, n_ties, ws, stream=None):
    _check(_lib.hmm_viterbi(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                            _ptr(path), _ptr(path_logp), _ptr(n_ties), _ptr(ws), _nbytes(ws),
                            _stream(stream)))


def hmm_posterior_decode(model, batch, prec, path, loglik, ws, stream=None):
    _check(_lib.hmm_posterior_decode(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                                     _ptr(path), _ptr(loglik), _ptr(ws), _nbytes(ws),
                                     _stream(stream)))


def default_mstep_opts(**kw) -> HmmMstepOptsC:
    o = HmmMstepOptsC()
    _lib.hmm_mstep_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def hmm_mstep_transitions(model, stats, opts, log_pi_out, log_A_out, stream=None):
    _check(_lib.hmm_mstep_transitions(ctypes.byref(model.c), _ptr(stats),
                                      None if opts is None else ctypes.byref(opts),
                                      _ptr(log_pi_out), _ptr(log_A_out), _stream(stream)))


MSTEP_NAMES = {"gaussian": "hmm_mstep_gaussian", "gamma": "hmm_mstep_gamma",
               "student_t": "hmm_mstep_student_t", "poisson": "hmm_mstep_poisson",
               "diag": "hmm_mstep_diag_gaussian", "full": "hmm_mstep_full_gaussian"}


def hmm_mstep(model, stats, opts, theta_out, collapsed=None, iters=None, stream=None):
    """Calls hmm_mstep_<family> for the model's family."""
    fn = getattr(_lib, MSTEP_NAMES[model.family])
    _check(fn(ctypes.byref(model.c), _ptr(stats), None if opts is None else ctypes.byref(opts),
              _ptr(theta_out), _ptr(collapsed), _ptr(iters), _stream(stream)))


def em_iteration(model, batch, prec, stats, loglik, status, ws, opts=None, stream=None):
    """One Baum-Welch iteration, in place on the device: E-step into `stats`,
    then the transition and emission M-steps overwrite the model tensors."""
    hmm_estep_stats(model, batch, prec, stats, loglik, status, ws, stream)
    hmm_mstep_transitions(model, stats, opts, model.log_pi, model.log_A, stream)
    hmm_mstep(model, stats, opts, model.theta, None, None, stream)


def hmm_set_chunk_len(steps: int):
    _check(_lib.hmm_set_chunk_len(int(steps)))


def hmm_autotune(model, batch, prec, stats, loglik, seq_status, ws, stream=None):
    """Times every variant of the call's route and keeps the fastest; returns
    (variant, [median ms of each variant])."""
    v = ctypes.c_int32(-1)
    ms = (ctypes.c_float * 4)()
    _check(_lib.hmm_autotune(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                             _ptr(stats), _ptr(loglik), _ptr(seq_status), _ptr(ws), _nbytes(ws),
                             _stream(stream), ctypes.byref(v), ms))
    n = ctypes.c_int32(0)
    _check(_lib.hmm_get_variant(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec], None,
                                ctypes.byref(n)))
    return int(v.value), [float(ms[k]) for k in range(n.value)]


def hmm_set_variant(variant: int):
    _check(_lib.hmm_set_variant(int(variant)))


def hmm_get_variant(model, batch, prec):
    """(variant the next E-step takes, number of variants of its route)."""
    v, n = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.hmm_get_variant(ctypes.byref(model.c), ctypes.byref(batch.c), PREC[prec],
                                ctypes.byref(v), ctypes.byref(n)))
    return int(v.value), int(n.value)


def hmm_profile_enable(on: bool):
    _check(_lib.hmm_profile_enable(1 if on else 0))


def hmm_profile_reset():
    _check(_lib.hmm_profile_reset())


def hmm_profile_records():
    """[(kernel name, milliseconds)] of the kernels recorded since the last reset."""
    out = []
    for i in range(_lib.hmm_profile_count()):
        name = ctypes.c_char_p()
        ms = ctypes.c_float()
        _check(_lib.hmm_profile_get(i, ctypes.byref(name), ctypes.byref(ms)))
        out.append((name.value.decode(), ms.value))
    return out


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def _ws(nbytes):
    import torch
    # torch's caching allocator returns 256-byte aligned blocks
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


# --------------------------------------------------------------------------
# helpers that allocate outputs
# --------------------------------------------------------------------------

def _rdtype(prec):
    import torch
    return torch.float64 if prec in ("f64", "plain_f64") else torch.float32


def estep_stats(model: DeviceModel, batch: DeviceBatch, prec="f32", ws=None, stream=None):
    import torch
    S = hmm_stats_len(model)
    stats = torch.empty(S, dtype=torch.float64, device="cuda")
    loglik = torch.empty(max(batch.n_seq, 1), dtype=torch.float64, device="cuda")
    status = torch.empty(max(batch.n_seq, 1), dtype=torch.int32, device="cuda")
    if ws is None:
        ws = _ws(hmm_workspace_size("estep", model, batch, prec))
    hmm_estep_stats(model, batch, prec, stats, loglik, status, ws, stream)
    return stats, loglik[:batch.n_seq], status[:batch.n_seq]


def forward_backward(model, batch, prec="f32", want_gamma=True, ws=None, stream=None):
    import torch
    loglik = torch.empty(max(batch.n_seq, 1), dtype=torch.float64, device="cuda")
    status = torch.empty(max(batch.n_seq, 1), dtype=torch.int32, device="cuda")
    gamma = torch.empty((max(batch.total, 1), model.n_states), dtype=_rdtype(prec),
                        device="cuda") if want_gamma else None
    if ws is None:
        ws = _ws(hmm_workspace_size("forward_backward", model, batch, prec))
    hmm_forward_backward(model, batch, prec, loglik, gamma, status, ws, stream)
    g = gamma[:batch.total] if gamma is not None else None
    return loglik[:batch.n_seq], g, status[:batch.n_seq]


def emission_logpdf(model, batch, prec="f32", ws=None, stream=None):
    import torch
    out = torch.empty((max(batch.total, 1), model.n_states), dtype=_rdtype(prec), device="cuda")
    if ws is None:
        ws = _ws(hmm_workspace_size("emission", model, batch, prec))
    hmm_emission_logpdf(model, batch, prec, out, ws, stream)
    return out[:batch.total]


def viterbi(model, batch, prec="f64", ws=None, stream=None):
    """Returns (path [sum T] int32, path log-probability [B] float64,
    near-ties met along each path [B] int32)."""
    import torch
    path = torch.empty(max(batch.total, 1), dtype=torch.int32, device="cuda")
    logp = torch.empty(max(batch.n_seq, 1), dtype=torch.float64, device="cuda")
    ties = torch.empty(max(batch.n_seq, 1), dtype=torch.int32, device="cuda")
    if ws is None:
        ws = _ws(hmm_workspace_size("viterbi", model, batch, prec))
    hmm_viterbi(model, batch, prec, path, logp, ties, ws, stream)
    return path[:batch.total], logp[:batch.n_seq], ties[:batch.n_seq]


def posterior_decode(model, batch, prec="f32", ws=None, stream=None):
    import torch
    path = torch.empty(max(batch.total, 1), dtype=torch.int32, device="cuda")
    loglik = torch.empty(max(batch.n_seq, 1), dtype=torch.float64, device="cuda")
    if ws is None:
        ws = _ws(hmm_workspace_size("posterior_decode", model, batch, prec))
    hmm_posterior_decode(model, batch, prec, path, loglik, ws, stream)
    return path[:batch.total], loglik[:batch.n_seq]


# --------------------------------------------------------------------------
# serving runtime (include/hmm_serve.h)
# --------------------------------------------------------------------------

def hmm_server_default_opts() -> HmmServerOptsC:
    o = HmmServerOptsC()
    _lib.hmm_server_default_opts(ctypes.byref(o))
    return o


def hmm_server_now() -> float:
    return _lib.hmm_server_now()


class Server:
    """Owns one hmm_server.  Models are registered from DeviceModel objects;
    submit() takes host observations and a host int32 path buffer that the
    server fills before the request's completion is returned by poll()."""

    def __init__(self, hbm_budget=None, host_staging=None, max_batch=None, n_streams=None,
                 prec="f32", device=0):
        o = hmm_server_default_opts()
        if hbm_budget is not None:
            o.hbm_budget = int(hbm_budget)
        if host_staging is not None:
            o.host_staging = int(host_staging)
        if max_batch is not None:
            o.max_batch = int(max_batch)
        if n_streams is not None:
            o.n_streams = int(n_streams)
        o.precision = PREC[prec]
        o.device = int(device)
        h = ctypes.c_void_p()
        _check(_lib.hmm_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._bufs = {}      # id -> (path buffer, obs copy kept for the caller's convenience)
        self.opts = o

    def add_model(self, model: "DeviceModel") -> int:
        mid = ctypes.c_int32()
        _check(_lib.hmm_server_add_model(self._h, ctypes.byref(model.c), ctypes.byref(mid)))
        return mid.value

    def submit(self, model_id: int, kind: str, obs, path_out: Optional[np.ndarray] = None):
        obs = np.ascontiguousarray(obs)
        f64 = obs.dtype == np.float64
        if not f64:
            obs = np.ascontiguousarray(obs, dtype=np.float32)
        T = int(obs.shape[0])
        if path_out is None:
            path_out = np.empty(T, dtype=np.int32)
        assert path_out.dtype == np.int32 and path_out.flags.c_contiguous and path_out.size >= T
        rid = ctypes.c_uint64()
        _check(_lib.hmm_server_submit(self._h, int(model_id), REQ[kind],
                                      obs.ctypes.data_as(ctypes.c_void_p), 1 if f64 else 0, T,
                                      path_out.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(rid)))
        self._bufs[rid.value] = path_out
        return rid.value

    def poll(self, max_n=256, timeout_us=0):
        arr = (HmmCompletionC * max_n)()
        n = ctypes.c_int32()
        _check(_lib.hmm_server_poll(self._h, arr, int(max_n), int(timeout_us), ctypes.byref(n)))
        out = []
        for i in range(n.value):
            c = arr[i]
            out.append({"id": c.id, "model": c.model, "kind": c.kind, "status": c.status,
                        "batch_size": c.batch_size, "T": c.T, "logp": c.logp,
                        "t_submit": c.t_submit, "t_launch": c.t_launch, "t_done": c.t_done,
                        "path": self._bufs.pop(c.id, None)})
        return out

    def info(self):
        i = HmmServerInfoC()
        _check(_lib.hmm_server_get_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in HmmServerInfoC._fields_}

    def close(self):
        if self._h:
            _check(_lib.hmm_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
