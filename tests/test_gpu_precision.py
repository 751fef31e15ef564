"""Scaled low-precision recursions (bf16 / fp16 matrix-core products with
FP32 accumulation and per-step rescaling) against the FP64 oracle.

These paths are approximations by construction: the test states their
error per output (log-likelihood, posteriors, pooled statistics) and checks
it against bounds set from the unit roundoff of the operand format (bf16
2^-9, fp16 2^-12) with a margin, plus the identities that per-step
normalisation keeps whatever the rounding (posteriors sum to one, so the
gamma totals count the steps).  The xi normaliser is the forward product,
which the low-precision path rounds, so the xi total (T - B exactly in
FP32/FP64) is only held to the format's statistics bound.  The printed
figures are the precision study's numbers.
"""
import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads

pytestmark = pytest.mark.gpu

# bounds per format: (log-likelihood relative, gamma absolute, statistics
# relative to their natural scale)
BOUNDS = {"bf16_scaled": (2e-3, 0.08, 0.05), "f16_scaled": (3e-4, 0.02, 0.01),
          "f32": (1e-4, 1e-4, 1e-4), "f64": (1e-10, 1e-9, 1e-9)}


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_29208_amd as h
    return h


def errors(h, w, prec):
    import torch
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
    stats, ll, st = h.estep_stats(dm, db, prec)
    llg, gam, _ = h.forward_backward(dm, db, prec)
    torch.cuda.synchronize()
    ref = oracle.estep(w.model, w.offsets, w.obs, want_gamma=True)
    s = stats.cpu().numpy()
    rs = ref["stats"]
    ll = ll.cpu().numpy()
    g = gam.cpu().numpy().astype(np.float64)
    n = w.model.n_states
    e_ll = float(np.max(np.abs(ll - ref["loglik"]) / np.abs(ref["loglik"])))
    e_g = float(np.max(np.abs(g - ref["gamma"])))
    # pooled statistics: each block relative to its own scale
    blocks = {"gamma1": slice(1, 1 + n), "xi": slice(1 + n, 1 + n + n * n),
              "gamma_sum": slice(1 + n + n * n, 1 + 2 * n + n * n),
              "family": slice(1 + 2 * n + n * n, None)}
    e_s = {k: float(np.max(np.abs(s[v] - rs[v])) / max(np.max(np.abs(rs[v])), 1e-300))
           for k, v in blocks.items()}
    return e_ll, e_g, e_s, g, s


@pytest.mark.parametrize("prec", ["bf16_scaled", "f16_scaled", "f32"])
@pytest.mark.parametrize("fam,n,d", [("gaussian", 20, 1), ("student_t", 64, 1),
                                     ("diag", 256, 16), ("gamma", 130, 1)])
def test_scaled_precision_error(h, prec, fam, n, d):
    w = workloads.random_workload(fam, n, d, [1, 64, 300, 700], 900 + n)
    e_ll, e_g, e_s, g, s = errors(h, w, prec)
    print(f"\n[precision] {prec:12s} {fam:9s} N={n:3d} D={d:2d}: loglik rel {e_ll:.2e}, "
          f"gamma abs {e_g:.2e}, stats rel " + ", ".join(f"{k} {v:.2e}" for k, v in e_s.items()))
    b_ll, b_g, b_s = BOUNDS[prec]
    assert e_ll <= b_ll and e_g <= b_g
    assert max(e_s.values()) <= b_s
    # identities that rounding does not break: sum_j gamma_t(j) = 1 per step
    assert np.allclose(g.sum(axis=1), 1.0, atol=1e-5)
    N = n
    xi = s[1 + N:1 + N + N * N].reshape(N, N)
    gs = s[1 + N + N * N:1 + 2 * N + N * N]
    T = int(w.offsets[-1])
    assert abs(gs.sum() - T) < 1e-4 * T
    assert abs(xi.sum() - (T - (len(w.offsets) - 1))) < b_s * T


def test_config3_precision_study(h):
    """Large-state workload (N = 256, D = 16), three sequences of 2048 steps:
    every precision's error against the oracle, printed side by side."""
    w = workloads.config3(n_seq=3)
    for prec in ("f64", "f32", "bf16_scaled", "f16_scaled"):
        e_ll, e_g, e_s, _, _ = errors(h, w, prec)
        print(f"\n[precision] config3 {prec:12s}: loglik rel {e_ll:.2e}, gamma abs {e_g:.2e}, "
              "stats rel " + ", ".join(f"{k} {v:.2e}" for k, v in e_s.items()))
        b_ll, b_g, b_s = BOUNDS[prec]
        assert e_ll <= b_ll and e_g <= b_g and max(e_s.values()) <= b_s


@pytest.mark.parametrize("prec", ["bf16_scaled", "f16_scaled"])
@pytest.mark.parametrize("n", [96, 193])
def test_scaled_many_groups(h, prec, n):
    """Thirty-seven sequences of mixed lengths (1 to 400 steps): the scaled
    sweeps step sixteen sequences per workgroup, so this spans two full
    groups, a partial third one and members that end long before the
    group's longest; every sequence must meet the same bounds."""
    rng = np.random.default_rng(77 + n)
    lengths = [1, 2, 400] + [int(x) for x in rng.integers(1, 260, size=34)]
    w = workloads.random_workload("gaussian", n, 1, lengths, 3100 + n)
    e_ll, e_g, e_s, g, s = errors(h, w, prec)
    print(f"\n[precision] {prec:12s} 37 sequences N={n}: loglik rel {e_ll:.2e}, gamma abs "
          f"{e_g:.2e}, stats rel " + ", ".join(f"{k} {v:.2e}" for k, v in e_s.items()))
    b_ll, b_g, b_s = BOUNDS[prec]
    assert e_ll <= b_ll and e_g <= b_g
    assert max(e_s.values()) <= b_s
    assert np.allclose(g.sum(axis=1), 1.0, atol=1e-5)


@pytest.mark.parametrize("prec", ["bf16_scaled", "f16_scaled"])
def test_scaled_status_codes_and_exclusion(h, prec):
    """A non-finite observation (status 2) and one outside the Gamma support
    (status 1) inside one group of the scaled sweeps: those two sequences
    get zero posteriors and add nothing to the statistics; the other two
    meet the format's bounds."""
    import torch
    w = workloads.random_workload("gamma", 80, 1, [50, 60, 70, 33], 860)
    obs = w.obs.copy()
    obs[w.offsets[1] + 5] = np.nan
    obs[w.offsets[2] + 40] = -1.0
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(obs, w.offsets, dtype=np.float32)
    stats, ll, st = h.estep_stats(dm, db, prec)
    llg, gam, st2 = h.forward_backward(dm, db, prec)
    torch.cuda.synchronize()
    ref = oracle.estep(w.model, w.offsets, obs, want_gamma=True)
    assert list(st.cpu().numpy()) == list(st2.cpu().numpy()) == list(ref["status"]) == [0, 2, 1, 0]
    ll = ll.cpu().numpy()
    assert ll[2] == -np.inf and np.isnan(ll[1])
    b_ll, b_g, b_s = BOUNDS[prec]
    ok = [0, 3]
    rl = ref["loglik"][ok]
    assert np.max(np.abs(ll[ok] - rl) / np.abs(rl)) <= b_ll
    g = gam.cpu().numpy().astype(np.float64)
    o = w.offsets
    assert not g[o[1]:o[3]].any()
    rows = np.r_[o[0]:o[1], o[3]:o[4]]
    assert np.max(np.abs(g[rows] - ref["gamma"][rows])) <= b_g
    s, rs = stats.cpu().numpy(), ref["stats"]
    n = w.model.n_states
    for sl in (slice(1, 1 + n), slice(1 + n, 1 + n + n * n), slice(1 + n + n * n, 1 + 2 * n + n * n)):
        assert np.max(np.abs(s[sl] - rs[sl])) <= b_s * max(np.max(np.abs(rs[sl])), 1e-300)
