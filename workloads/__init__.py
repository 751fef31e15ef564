"""Seeded synthetic workloads for the HMM E-step.

This module only draws random inputs: model parameters, sequence lengths,
hidden state paths and observations.  It holds none of the inference
arithmetic (no emission densities, recursions or statistics), so both the
CPU oracle and the GPU library can consume what it produces.

Every draw comes from ``numpy.random.default_rng(seed)`` (PCG64) with
``seed = 1000 * config + replicate``.  Draw order: parameters, then lengths,
then the state paths (all sequences advanced together one time step at a
time), then the observations given the states.

Model layout (shared with the C ABI):
    log_pi [N]           log initial probabilities
    log_A  [N, N]        log transition probabilities, row i = from state i
    theta  flat float64  family parameters, structure-of-arrays over states:
        gaussian     [mu(N), var(N)]
        gamma        [shape(N), rate(N)]          (rate = 1 / scale)
        student_t    [mu(N), sigma(N), nu(N)]
        poisson      [lambda(N)]
        diag         [mu(N*D), var(N*D)]
        full         [mu(N*D), L(N*D*D)]           (lower Cholesky, row-major)

The workload families mirror the paper's benchmark domains (paper section 6:
animal movement step lengths -> Gamma, financial returns -> Student-t,
counts -> Poisson, multivariate returns -> full covariance), scaled up; the
paper's own datasets are not used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

FAMILIES = ("gaussian", "gamma", "student_t", "poisson", "diag", "full")
SCALAR_FAMILIES = ("gaussian", "gamma", "student_t", "poisson")


@dataclasses.dataclass
class Model:
    family: str
    n_states: int
    dim: int
    log_pi: np.ndarray      # [N] float64
    log_A: np.ndarray       # [N, N] float64
    theta: np.ndarray       # flat float64

    def copy(self) -> "Model":
        return Model(self.family, self.n_states, self.dim, self.log_pi.copy(),
                     self.log_A.copy(), self.theta.copy())


@dataclasses.dataclass
class Workload:
    name: str
    model: Model
    lengths: np.ndarray     # [B] int64
    offsets: np.ndarray     # [B+1] int64
    obs: np.ndarray         # [sum T, D] float64 (D = 1 -> shape [sum T, 1])
    states: np.ndarray      # [sum T] int32, the simulated hidden path

    @property
    def n_seq(self) -> int:
        return int(self.lengths.shape[0])

    @property
    def total_steps(self) -> int:
        return int(self.offsets[-1])

    @property
    def transitions(self) -> int:
        """Sum over sequences of T_b * N^2 (the throughput unit)."""
        n = self.model.n_states
        return int(self.lengths.sum()) * n * n

    def obs32(self) -> np.ndarray:
        return self.obs.astype(np.float32)

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(lens)
        obs = np.concatenate([self.obs[self.offsets[b]:self.offsets[b + 1]] for b in idx]) \
            if len(idx) else self.obs[:0]
        st = np.concatenate([self.states[self.offsets[b]:self.offsets[b + 1]] for b in idx]) \
            if len(idx) else self.states[:0]
        return Workload(self.name + "[sub]", self.model, lens, offs, obs, st)


# --------------------------------------------------------------------------
# parameter draws
# --------------------------------------------------------------------------

def _sticky_rows(rng, n, diag, conc=1.0):
    """Rows with `diag` on the diagonal and (1-diag)*Dirichlet(conc) spread
    over the off-diagonal entries."""
    A = np.zeros((n, n))
    if n == 1:
        A[0, 0] = 1.0
        return A
    for i in range(n):
        off = rng.dirichlet(np.full(n - 1, conc))
        row = np.insert(off * (1.0 - diag), i, diag)
        A[i] = row
    return A


def _haar_orthogonal(rng, d):
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    return q


def _logs(p):
    with np.errstate(divide="ignore"):
        return np.log(p)


def make_model(family, n, d=1, rng=None, *, sticky=0.9, off_conc=1.0,
               mix_rows=None) -> Model:
    """Draw a random model of the given family and size."""
    rng = rng if rng is not None else np.random.default_rng(0)
    if mix_rows is not None:
        # A_i = w e_i + (1 - w) Dirichlet(mix_rows * 1_N)
        w = 0.5
        A = np.stack([w * np.eye(n)[i] + (1 - w) * rng.dirichlet(np.full(n, mix_rows))
                      for i in range(n)])
    else:
        A = _sticky_rows(rng, n, sticky, off_conc)
    pi = np.full(n, 1.0 / n)
    if family == "gaussian":
        mu = rng.normal(0.0, 2.0, n)
        var = rng.uniform(0.5, 2.0, n)
        theta = np.concatenate([mu, var])
    elif family == "gamma":
        shape = rng.uniform(1.0, 10.0, n)
        scale = rng.uniform(0.5, 3.0, n)
        theta = np.concatenate([shape, 1.0 / scale])
    elif family == "student_t":
        mu = rng.normal(0.0, 2.0, n)
        sig = rng.uniform(0.5, 2.0, n)
        nu = rng.uniform(2.0, 30.0, n)
        theta = np.concatenate([mu, sig, nu])
    elif family == "poisson":
        lam = np.sort(rng.uniform(1.0, 100.0, n))
        theta = lam.copy()
    elif family == "diag":
        mu = rng.normal(0.0, 2.0, (n, d))
        var = rng.uniform(0.5, 2.0, (n, d))
        theta = np.concatenate([mu.ravel(), var.ravel()])
    elif family == "full":
        mu = rng.normal(0.0, 2.0, (n, d))
        Ls = []
        for _ in range(n):
            q = _haar_orthogonal(rng, d)
            lam = np.exp(rng.uniform(math.log(1e-3), 0.0, d))
            if d > 1:   # pin the spectrum ends so the condition number is exactly 1e3
                lam[0], lam[-1] = 1.0, 1e-3
            sig = (q * lam[None, :]) @ q.T
            sig = 0.5 * (sig + sig.T)
            Ls.append(np.linalg.cholesky(sig))
        theta = np.concatenate([mu.ravel(), np.stack(Ls).ravel()])
    else:
        raise ValueError(f"unknown family {family!r}")
    return Model(family, n, d if family in ("diag", "full") else 1,
                 _logs(pi), _logs(A), theta.astype(np.float64))


# --------------------------------------------------------------------------
# simulation
# --------------------------------------------------------------------------

def simulate_states(rng, model: Model, lengths) -> np.ndarray:
    """All sequences advance one step at a time (inverse-CDF sampling)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    B = len(lengths)
    offs = np.zeros(B + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)
    out = np.zeros(int(offs[-1]), dtype=np.int32)
    if B == 0:
        return out
    pi = np.exp(model.log_pi)
    cpi = np.cumsum(pi)
    cpi[-1] = 1.0 + 1e-12
    cA = np.cumsum(np.exp(model.log_A), axis=1)
    cA[:, -1] = 1.0 + 1e-12
    n = model.n_states
    Tmax = int(lengths.max())
    cur = np.searchsorted(cpi, rng.random(B), side="right").clip(0, n - 1)
    active = lengths > 0
    out[offs[:-1][active]] = cur[active]
    for t in range(1, Tmax):
        u = rng.random(B)
        rows = cA[cur]
        nxt = (u[:, None] >= rows).sum(axis=1).clip(0, n - 1)
        cur = nxt
        alive = lengths > t
        out[offs[:-1][alive] + t] = cur[alive]
    return out


def simulate_obs(rng, model: Model, states: np.ndarray) -> np.ndarray:
    n, d = model.n_states, model.dim
    th = model.theta
    s = states
    m = len(s)
    if model.family == "gaussian":
        mu, var = th[:n], th[n:2 * n]
        y = rng.normal(mu[s], np.sqrt(var[s]))
        return y.reshape(m, 1)
    if model.family == "gamma":
        shape, rate = th[:n], th[n:2 * n]
        y = rng.gamma(shape[s], 1.0 / rate[s])
        return y.reshape(m, 1)
    if model.family == "student_t":
        mu, sig, nu = th[:n], th[n:2 * n], th[2 * n:3 * n]
        y = mu[s] + sig[s] * rng.standard_t(nu[s])
        return y.reshape(m, 1)
    if model.family == "poisson":
        lam = th[:n]
        y = rng.poisson(lam[s]).astype(np.float64)
        return y.reshape(m, 1)
    if model.family == "diag":
        mu = th[:n * d].reshape(n, d)
        var = th[n * d:2 * n * d].reshape(n, d)
        return rng.normal(mu[s], np.sqrt(var[s]))
    if model.family == "full":
        mu = th[:n * d].reshape(n, d)
        L = th[n * d:].reshape(n, d, d)
        z = rng.standard_normal((m, d))
        y = np.empty((m, d))
        for j in range(n):          # y_t = mu_j + L_j z_t for the steps in state j
            idx = np.nonzero(s == j)[0]
            y[idx] = mu[j] + z[idx] @ L[j].T
        return y
    raise ValueError(model.family)


def _offsets(lengths):
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)
    return offs


def simulate(name, model: Model, lengths, rng) -> Workload:
    lengths = np.asarray(lengths, dtype=np.int64)
    states = simulate_states(rng, model, lengths)
    obs = simulate_obs(rng, model, states)
    return Workload(name, model, lengths, _offsets(lengths), obs, states)


def lognormal_lengths(rng, b, median, sigma, lo, hi):
    z = rng.standard_normal(b)
    return np.clip(np.round(np.exp(math.log(median) + sigma * z)), lo, hi).astype(np.int64)


def perturb(model: Model, rng) -> Model:
    """Starting point for an EM iteration: the true parameters moved by a
    seeded perturbation (locations + 0.25 N(0,1), scales * exp(0.2 N(0,1)),
    transitions A <- A/2 + 1/(2N))."""
    m = model.copy()
    n, d = m.n_states, m.dim
    th = m.theta
    A = np.exp(m.log_A)
    A = 0.5 * A + 0.5 / n
    m.log_A = _logs(A / A.sum(axis=1, keepdims=True))
    if m.family == "gaussian":
        th[:n] += 0.25 * rng.standard_normal(n)
        th[n:2 * n] *= np.exp(0.2 * rng.standard_normal(n)) ** 2
    elif m.family == "gamma":
        th[:n] *= np.exp(0.2 * rng.standard_normal(n))
        th[n:2 * n] *= np.exp(0.2 * rng.standard_normal(n))
    elif m.family == "student_t":
        th[:n] += 0.25 * rng.standard_normal(n)
        th[n:2 * n] *= np.exp(0.2 * rng.standard_normal(n))
        th[2 * n:3 * n] *= np.exp(0.2 * rng.standard_normal(n))
    elif m.family == "poisson":
        th[:n] *= np.exp(0.2 * rng.standard_normal(n))
    elif m.family == "diag":
        th[:n * d] += 0.25 * rng.standard_normal(n * d)
        th[n * d:] *= np.exp(0.2 * rng.standard_normal(n * d)) ** 2
    elif m.family == "full":
        th[:n * d] += 0.25 * rng.standard_normal(n * d)
        L = th[n * d:].reshape(n, d, d)
        L *= np.exp(0.2 * rng.standard_normal(n))[:, None, None]
    m.theta = th
    return m


# --------------------------------------------------------------------------
# the five benchmark configurations
# --------------------------------------------------------------------------

def config1(replicate=0) -> Workload:
    """N=3 Gaussian (means -2, 0, 2, sd 1), a_ii = 0.9 with 0.1*Dirichlet(1)
    off the diagonal, uniform pi, one sequence of T = 1000."""
    rng = np.random.default_rng(1000 * 1 + replicate)
    n = 3
    A = _sticky_rows(rng, n, 0.9, 1.0)
    theta = np.concatenate([np.array([-2.0, 0.0, 2.0]), np.ones(n)])
    model = Model("gaussian", n, 1, _logs(np.full(n, 1.0 / n)), _logs(A), theta)
    return simulate("config1", model, [1000], rng)


def config2(replicate=0, n_seq=1024) -> Workload:
    """B = 1024 ragged sequences, T_b ~ U{500..5000}, N = 8 Gamma states
    (shape U[1,10], scale U[0.5,3]), a_ii = 0.95."""
    rng = np.random.default_rng(1000 * 2 + replicate)
    n = 8
    A = _sticky_rows(rng, n, 0.95, 1.0)
    shape = rng.uniform(1.0, 10.0, n)
    scale = rng.uniform(0.5, 3.0, n)
    model = Model("gamma", n, 1, _logs(np.full(n, 1.0 / n)), _logs(A),
                  np.concatenate([shape, 1.0 / scale]))
    lengths = rng.integers(500, 5000, size=n_seq, endpoint=True)
    return simulate("config2", model, lengths, rng)


def config3(replicate=0, n_seq=256, T=2048) -> Workload:
    """N = 256 diagonal-Gaussian states, D = 16, B = 256 sequences of
    T = 2048; A_i = 0.5 e_i + 0.5 Dirichlet(0.5)."""
    rng = np.random.default_rng(1000 * 3 + replicate)
    n, d = 256, 16
    A = np.stack([0.5 * np.eye(n)[i] + 0.5 * rng.dirichlet(np.full(n, 0.5)) for i in range(n)])
    mu = rng.normal(0.0, 2.0, (n, d))
    var = rng.uniform(0.5, 2.0, (n, d))
    model = Model("diag", n, d, _logs(np.full(n, 1.0 / n)), _logs(A),
                  np.concatenate([mu.ravel(), var.ravel()]))
    return simulate("config3", model, np.full(n_seq, T), rng)


def config4a(replicate=0, n_seq=512) -> Workload:
    """N = 32 full-covariance Gaussian states in D = 32 (condition number
    1e3), B = 512 log-normal lengths (median 3000, sigma 0.6, <= 20000)."""
    rng = np.random.default_rng(1000 * 4 + replicate)
    n, d = 32, 32
    model = make_model("full", n, d, rng, sticky=0.9)
    lengths = lognormal_lengths(rng, n_seq, 3000, 0.6, 16, 20000)
    return simulate("config4a", model, lengths, rng)


def config4b(replicate=0, n_seq=512) -> Workload:
    """N = 32 scalar Student-t states (nu ~ U[2,30]), same length law."""
    rng = np.random.default_rng(1000 * 4 + 500 + replicate)
    n = 32
    model = make_model("student_t", n, 1, rng, sticky=0.9)
    lengths = lognormal_lengths(rng, n_seq, 3000, 0.6, 16, 20000)
    return simulate("config4b", model, lengths, rng)


def serving_models(replicate=0):
    """Sixteen resident models: 6 with N=4, 5 with N=16, 5 with N=64,
    alternating Gaussian and Poisson emissions."""
    rng = np.random.default_rng(1000 * 5 + replicate)
    sizes = [4] * 6 + [16] * 5 + [64] * 5
    models = []
    for k, n in enumerate(sizes):
        fam = "gaussian" if k % 2 == 0 else "poisson"
        models.append(make_model(fam, n, 1, rng, sticky=0.9))
    return models


def serving_request_lengths(rng, count, median=2000, sigma=1.0, lo=16, hi=100000):
    return lognormal_lengths(rng, count, median, sigma, lo, hi)


def random_workload(family, n, d, lengths, seed) -> Workload:
    """Small seeded workload for parity and property tests."""
    rng = np.random.default_rng(seed)
    model = make_model(family, n, d, rng)
    return simulate(f"{family}-N{n}-D{d}-s{seed}", model, lengths, rng)


CONFIGS = {
    "config1": config1,
    "config2": config2,
    "config3": config3,
    "config4a": config4a,
    "config4b": config4b,
}
