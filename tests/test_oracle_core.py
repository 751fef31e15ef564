"""Pins for the FP64 oracle's inference half (emission, forward-backward,
posteriors, pooled statistics, Viterbi, posterior decoding).

Each check compares the oracle with something that is not the oracle:
brute-force enumeration of all N^T paths, scipy's densities, numerical
quadrature, closed forms of special models, or identities of the exact
posteriors (section 3.1 definitions).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
import workloads
from tests.brute import brute_posteriors, brute_viterbi


def rand_model(rng, n, asym=True):
    A = rng.dirichlet(np.ones(n), size=n)
    pi = rng.dirichlet(np.ones(n))
    return np.log(pi), np.log(A)


# ----------------------------------------------------------------- emission

def test_emission_gaussian_vs_scipy():
    rng = np.random.default_rng(1)
    n = 4
    mu, var = rng.normal(0, 2, n), rng.uniform(0.3, 3, n)
    y = rng.normal(0, 3, 50)
    out = oracle.emission("gaussian", n, 1, np.concatenate([mu, var]), y)
    ref = stats.norm.logpdf(y[:, None], mu[None], np.sqrt(var)[None])
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_emission_gamma_vs_scipy_and_support():
    rng = np.random.default_rng(2)
    n = 5
    a, b = rng.uniform(0.5, 10, n), rng.uniform(0.2, 3, n)
    y = rng.gamma(2.0, 2.0, 40)
    out = oracle.emission("gamma", n, 1, np.concatenate([a, b]), y)
    ref = stats.gamma.logpdf(y[:, None], a[None], scale=1.0 / b[None])
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)
    bad = oracle.emission("gamma", n, 1, np.concatenate([a, b]), np.array([0.0, -1.0]))
    assert np.all(bad == -np.inf)


def test_emission_student_t_vs_scipy():
    rng = np.random.default_rng(3)
    n = 4
    mu, s, nu = rng.normal(0, 2, n), rng.uniform(0.5, 2, n), rng.uniform(1.5, 40, n)
    y = rng.standard_t(3, 60) * 2
    out = oracle.emission("student_t", n, 1, np.concatenate([mu, s, nu]), y)
    ref = stats.t.logpdf(y[:, None], nu[None], loc=mu[None], scale=s[None])
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_emission_poisson_vs_scipy_and_support():
    lam = np.array([0.5, 3.0, 40.0])
    y = np.array([0, 1, 2, 7, 30, 55], dtype=np.float64)
    out = oracle.emission("poisson", 3, 1, lam, y)
    ref = stats.poisson.logpmf(y[:, None].astype(int), lam[None])
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)
    bad = oracle.emission("poisson", 3, 1, lam, np.array([2.5, -1.0]))
    assert np.all(bad == -np.inf)


def test_emission_diag_vs_scipy():
    rng = np.random.default_rng(4)
    n, d = 3, 5
    mu, var = rng.normal(0, 2, (n, d)), rng.uniform(0.5, 2, (n, d))
    y = rng.normal(0, 2, (20, d))
    out = oracle.emission("diag", n, d, np.concatenate([mu.ravel(), var.ravel()]), y)
    ref = np.stack([stats.multivariate_normal.logpdf(y, mu[j], np.diag(var[j])) for j in range(n)], 1)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-11)


def test_emission_full_vs_scipy():
    rng = np.random.default_rng(5)
    m = workloads.make_model("full", 3, 6, rng)
    y = rng.normal(0, 2, (25, 6))
    out = oracle.emission("full", 3, 6, m.theta, y)
    mu = m.theta[:18].reshape(3, 6)
    L = m.theta[18:].reshape(3, 6, 6)
    ref = np.stack([stats.multivariate_normal.logpdf(y, mu[j], L[j] @ L[j].T) for j in range(3)], 1)
    np.testing.assert_allclose(out, ref, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("family,theta", [
    ("gaussian", [0.7, 1.9]),
    ("gamma", [3.5, 1.7]),
    ("student_t", [0.3, 1.4, 4.5]),
])
def test_emission_integrates_to_one(family, theta):
    f = lambda v: math.exp(oracle.emission(family, 1, 1, np.array(theta), np.array([v]))[0, 0])
    lo = 0.0 if family == "gamma" else -np.inf
    val, _ = integrate.quad(f, lo, np.inf, limit=400)
    assert abs(val - 1.0) < 1e-8


def test_poisson_sums_to_one():
    lp = oracle.emission("poisson", 1, 1, np.array([7.3]), np.arange(200.0))
    assert abs(np.exp(lp).sum() - 1.0) < 1e-12


def test_full_d1_reduces_to_gaussian():
    y = np.array([-1.3, 0.2, 2.5])
    full = oracle.emission("full", 2, 1, np.array([0.5, -1.0, 1.3, 0.7]), y)
    gau = oracle.emission("gaussian", 2, 1, np.array([0.5, -1.0, 1.3 ** 2, 0.7 ** 2]), y)
    np.testing.assert_allclose(full, gau, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------- lse

def test_lse_definition_and_all_neg_inf():
    x = np.array([-1000.0, -1001.0, -999.5])
    assert abs(oracle.lse(x) - special.logsumexp(x)) < 1e-12
    assert oracle.lse(np.array([-np.inf, -np.inf])) == -np.inf
    assert oracle.lse(np.array([-np.inf, 2.0])) == 2.0


# ------------------------------------------------------- forward-backward

@pytest.mark.parametrize("n,T,seed", [(2, 1, 0), (2, 9, 1), (3, 7, 2), (3, 5, 3), (2, 14, 4)])
def test_forward_backward_vs_brute_force(n, T, seed):
    rng = np.random.default_rng(seed)
    log_pi, log_A = rand_model(rng, n)
    logB = rng.normal(-1.0, 1.5, (T, n))
    alpha = oracle.forward(log_pi, log_A, logB)
    beta = oracle.backward(log_A, logB)
    ll = oracle.lse(alpha[-1])
    ll_b = oracle.lse(log_pi + logB[0] + beta[0])
    gamma, xi, xs = oracle.posteriors(log_A, logB, alpha, beta, ll)
    bl, bg, bx = brute_posteriors(log_pi, log_A, logB)
    assert abs(ll - bl) <= 1e-12 * abs(bl) + 1e-13
    assert abs(ll_b - bl) <= 1e-12 * abs(bl) + 1e-13
    np.testing.assert_allclose(gamma, bg, rtol=1e-11, atol=1e-14)
    if T > 1:
        np.testing.assert_allclose(xi, bx, rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(xs, bx.sum(0), rtol=1e-11, atol=1e-14)


def test_forward_backward_with_structural_zeros():
    rng = np.random.default_rng(7)
    n, T = 3, 6
    A = np.array([[0.5, 0.5, 0.0], [0.0, 0.3, 0.7], [0.6, 0.0, 0.4]])
    log_A = np.log(np.where(A > 0, A, 1.0)) + np.where(A > 0, 0.0, -np.inf)
    log_pi = np.log(np.array([0.2, 0.3, 0.5]))
    logB = rng.normal(-1, 1, (T, n))
    alpha = oracle.forward(log_pi, log_A, logB)
    beta = oracle.backward(log_A, logB)
    ll = oracle.lse(alpha[-1])
    gamma, xi, _ = oracle.posteriors(log_A, logB, alpha, beta, ll)
    bl, bg, bx = brute_posteriors(log_pi, log_A, logB)
    assert abs(ll - bl) < 1e-12 * abs(bl)
    np.testing.assert_allclose(gamma, bg, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(xi, bx, rtol=1e-11, atol=1e-15)
    assert np.all(xi[:, A == 0] == 0)


def test_invariants_long_sequence():
    """sum_i gamma = 1; sum_j xi = gamma_t; sum_i xi = gamma_{t+1};
    forward and backward log-likelihoods agree (no underflow at T = 3000)."""
    w = workloads.random_workload("gamma", 5, 1, [3000], 11)
    m = w.model
    logB = oracle.emission("gamma", 5, 1, m.theta, w.obs)
    alpha = oracle.forward(m.log_pi, m.log_A, logB)
    beta = oracle.backward(m.log_A, logB)
    ll = oracle.lse(alpha[-1])
    ll_b = oracle.lse(m.log_pi + logB[0] + beta[0])
    assert np.isfinite(ll) and ll < -1000
    assert abs(ll - ll_b) <= 1e-12 * abs(ll)
    gamma, xi, _ = oracle.posteriors(m.log_A, logB, alpha, beta, ll)
    np.testing.assert_allclose(gamma.sum(1), 1.0, atol=1e-10)
    np.testing.assert_allclose(xi.sum(2), gamma[:-1], atol=1e-10)
    np.testing.assert_allclose(xi.sum(1), gamma[1:], atol=1e-10)


def test_single_state_closed_form():
    """N = 1: logL = sum_t log b(y_t), gamma = 1."""
    rng = np.random.default_rng(8)
    logB = rng.normal(-2, 1, (50, 1))
    alpha = oracle.forward(np.zeros(1), np.zeros((1, 1)), logB)
    assert abs(oracle.lse(alpha[-1]) - logB.sum()) < 1e-11


def test_iid_mixture_closed_form():
    """Identical rows a_ij = pi_j: the model is an i.i.d. mixture, so
    logL = sum_t lse_j(log pi_j + l_t(j)) and gamma_t are the responsibilities."""
    rng = np.random.default_rng(9)
    n, T = 4, 40
    pi = rng.dirichlet(np.ones(n))
    log_pi = np.log(pi)
    log_A = np.tile(log_pi, (n, 1))
    logB = rng.normal(-1, 2, (T, n))
    alpha = oracle.forward(log_pi, log_A, logB)
    beta = oracle.backward(log_A, logB)
    ll = oracle.lse(alpha[-1])
    mix = special.logsumexp(log_pi[None] + logB, axis=1)
    assert abs(ll - mix.sum()) < 1e-11 * abs(ll)
    gamma, _, _ = oracle.posteriors(log_A, logB, alpha, beta, ll)
    resp = np.exp(log_pi[None] + logB - mix[:, None])
    np.testing.assert_allclose(gamma, resp, rtol=1e-10, atol=1e-14)


def test_permutation_matrix_single_path():
    """A deterministic cycle with a known start admits one path: logL is its score."""
    n, T = 3, 10
    perm = [1, 2, 0]
    log_A = np.full((n, n), -np.inf)
    for i, j in enumerate(perm):
        log_A[i, j] = 0.0
    log_pi = np.array([0.0, -np.inf, -np.inf])
    rng = np.random.default_rng(10)
    logB = rng.normal(-1, 1, (T, n))
    alpha = oracle.forward(log_pi, log_A, logB)
    q, s = 0, 0.0
    for t in range(T):
        s += logB[t, q]
        q = perm[q]
    assert abs(oracle.lse(alpha[-1]) - s) < 1e-12


# ------------------------------------------------------------- pooled stats

def _family_terms(fam, model, y, j):
    n = model.n_states
    th = model.theta
    if fam == "gaussian":
        d = y[:, 0] - th[j]
        return np.stack([d, d * d], 1)
    if fam == "gamma":
        return np.stack([y[:, 0], np.log(y[:, 0]), y[:, 0] ** 2], 1)
    if fam == "poisson":
        return y[:, :1]
    if fam == "student_t":
        d = y[:, 0] - th[j]
        s, nu = th[n + j], th[2 * n + j]
        u = (nu + 1) / (nu + d * d / s ** 2)
        return np.stack([u, u * d, u * d * d, np.log(u) - u], 1)
    raise ValueError(fam)


@pytest.mark.parametrize("fam", ["gaussian", "gamma", "poisson", "student_t"])
def test_pooled_stats_vs_brute_force(fam):
    """Tiny batch: every statistic equals the brute-force posteriors reduced by numpy."""
    rng = np.random.default_rng(20)
    w = workloads.random_workload(fam, 3, 1, [5, 1, 6, 3], 21)
    m = w.model
    r = oracle.estep(m, w.offsets, w.obs)
    n = 3
    ll_sum = 0.0
    g1 = np.zeros(n)
    xs = np.zeros((n, n))
    gs = np.zeros(n)
    fb = np.zeros((n, len(_family_terms(fam, m, w.obs[:1], 0)[0])))
    for b in range(w.n_seq):
        y = w.obs[w.offsets[b]:w.offsets[b + 1]]
        logB = np.stack([stats_logpdf(fam, m, y, j) for j in range(n)], 1)
        bl, bg, bx = brute_posteriors(m.log_pi, m.log_A, logB)
        assert abs(r["loglik"][b] - bl) < 1e-11 * abs(bl)
        ll_sum += bl
        g1 += bg[0]
        xs += bx.sum(0)
        gs += bg.sum(0)
        for j in range(n):
            fb[j] += (bg[:, j:j + 1] * _family_terms(fam, m, y, j)).sum(0)
    s = r["stats"]
    ref = np.concatenate([[ll_sum], g1, xs.ravel(), gs, fb.ravel()])
    np.testing.assert_allclose(s, ref, rtol=1e-10, atol=1e-12)
    assert len(s) == oracle.stats_len(fam, n)


def stats_logpdf(fam, m, y, j):
    n = m.n_states
    th = m.theta
    if fam == "gaussian":
        return stats.norm.logpdf(y[:, 0], th[j], np.sqrt(th[n + j]))
    if fam == "gamma":
        return stats.gamma.logpdf(y[:, 0], th[j], scale=1 / th[n + j])
    if fam == "poisson":
        return stats.poisson.logpmf(y[:, 0].astype(int), th[j])
    if fam == "student_t":
        return stats.t.logpdf(y[:, 0], th[2 * n + j], loc=th[j], scale=th[n + j])
    raise ValueError(fam)


def test_pooled_stats_multivariate_vs_numpy():
    """diag and full blocks: gamma from the oracle reduced independently by numpy."""
    for fam, d in (("diag", 3), ("full", 3)):
        w = workloads.random_workload(fam, 3, d, [40, 17, 33], 30)
        m = w.model
        r = oracle.estep(m, w.offsets, w.obs, want_gamma=True)
        g = r["gamma"]
        n = 3
        mu = m.theta[:n * d].reshape(n, d)
        base = 1 + 2 * n + n * n
        K = 2 * d if fam == "diag" else d + d * (d + 1) // 2
        blk = r["stats"][base:].reshape(n, K)
        for j in range(n):
            dv = w.obs - mu[j]
            np.testing.assert_allclose(blk[j, :d], (g[:, j:j + 1] * dv).sum(0), rtol=1e-11, atol=1e-10)
            if fam == "diag":
                np.testing.assert_allclose(blk[j, d:], (g[:, j:j + 1] * dv * dv).sum(0), rtol=1e-11)
            else:
                S = (g[:, j, None, None] * dv[:, :, None] * dv[:, None, :]).sum(0)
                np.testing.assert_allclose(blk[j, d:], S[np.tril_indices(d)], rtol=1e-11, atol=1e-10)


def test_status_codes():
    w = workloads.random_workload("gamma", 3, 1, [5, 6, 4], 40)
    obs = w.obs.copy()
    obs[w.offsets[1] + 2] = np.nan           # sequence 1: non-finite observation
    obs[w.offsets[2] + 1] = -3.0             # sequence 2: outside the Gamma support
    r = oracle.estep(w.model, w.offsets, obs)
    assert list(r["status"]) == [0, 2, 1]
    assert r["loglik"][2] == -np.inf
    only0 = oracle.estep(w.model, w.offsets[:2], obs)
    np.testing.assert_allclose(r["stats"], only0["stats"], rtol=0, atol=0)


# ------------------------------------------------------------------- Viterbi

@pytest.mark.parametrize("n,T,seed", [(2, 12, 0), (3, 8, 1), (4, 6, 2), (3, 1, 3)])
def test_viterbi_vs_brute_force(n, T, seed):
    rng = np.random.default_rng(seed)
    log_pi, log_A = rand_model(rng, n)
    logB = rng.normal(-1, 1.5, (T, n))
    path, lp, ties = oracle.viterbi(log_pi, log_A, logB)
    bp, blp, _ = brute_viterbi(log_pi, log_A, logB)
    np.testing.assert_array_equal(path, bp)
    assert abs(lp - blp) < 1e-12 * max(1, abs(blp))
    assert ties == 0


def test_viterbi_tie_breaks_to_lowest_index():
    """Two exactly equal-scoring paths: the backtrace picks the lowest state."""
    n, T = 2, 4
    log_pi = np.log([0.5, 0.5])
    log_A = np.log([[0.5, 0.5], [0.5, 0.5]])
    logB = np.zeros((T, n))
    path, lp, ties = oracle.viterbi(log_pi, log_A, logB)
    assert list(path) == [0, 0, 0, 0]
    assert abs(lp - T * math.log(0.5)) < 1e-14
    assert ties == T


def test_posterior_decode_lowest_index():
    g = np.array([[0.2, 0.5, 0.3], [0.4, 0.4, 0.2], [0.1, 0.1, 0.8]])
    assert list(oracle.posterior_decode(g)) == [1, 0, 2]


# ----------------------------------------------------------------- workloads

def test_workloads_are_deterministic():
    a = workloads.config1()
    b = workloads.config1()
    assert np.array_equal(a.obs, b.obs) and np.array_equal(a.states, b.states)
    c = workloads.config2(n_seq=16)
    d = workloads.config2(n_seq=16)
    assert np.array_equal(c.obs, d.obs) and np.array_equal(c.lengths, d.lengths)
    assert c.lengths.min() >= 500 and c.lengths.max() <= 5000
    assert np.allclose(np.exp(c.model.log_A).sum(1), 1.0)
