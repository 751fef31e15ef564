"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances: 1e-9 relative for the FP64 paths, 1e-4 relative for the FP32
paths, on log-likelihoods and on the pooled statistics.

A statistic is compared relative to its natural scale,
|got - ref| <= tol * max(|ref|, s), where s is the size of the quantities it
is made of.  This matters only for sums that cancel:
  - shifted first moments sum g d (and sum g u d): s = sqrt(sum g * sum g d^2)
    (Cauchy-Schwarz bound of |sum g d|);
  - packed cross moments sum g d_r d_c: s = sqrt(sum g d_r^2 * sum g d_c^2);
  - sum g log y (Gamma): s = N_j (log y is of order one);
  - everything else: s = 1e-6 * max |block| (a floor against exact zeros).
"""
import numpy as np

TOL = {"f64": 1e-9, "plain_f64": 1e-9, "f32": 1e-4, "plain_f32": 1e-4}


def family_k(fam, d=1):
    return {"gaussian": 2, "gamma": 3, "student_t": 4, "poisson": 1, "diag": 2 * d,
            "full": d + d * (d + 1) // 2, "table": 0}[fam]


def natural_scale(ref, fam, N, d=1):
    ref = np.asarray(ref, dtype=np.float64)
    s = np.zeros_like(ref)
    blocks = [(0, 1), (1, 1 + N), (1 + N, 1 + N + N * N), (1 + N + N * N, 1 + 2 * N + N * N)]
    for a, b in blocks:
        s[a:b] = 1e-6 * np.max(np.abs(ref[a:b])) if b > a else 0
    K = family_k(fam, d)
    if K == 0:
        return s
    base = 1 + 2 * N + N * N
    gs = ref[1 + N + N * N:1 + 2 * N + N * N]
    F = ref[base:base + N * K].reshape(N, K)
    S = np.abs(F) * 1e-6 + 1e-6 * np.max(np.abs(F), axis=0, keepdims=True)
    if fam == "gaussian":
        S[:, 0] = np.sqrt(np.abs(gs * F[:, 1]))
    elif fam == "gamma":
        S[:, 1] = gs
    elif fam == "student_t":
        S[:, 1] = np.sqrt(np.abs(F[:, 0] * F[:, 2]))
    elif fam == "diag":
        S[:, :d] = np.sqrt(np.abs(gs[:, None] * F[:, d:]))
    elif fam == "full":
        diag_idx = [r * (r + 1) // 2 + r for r in range(d)]
        second = F[:, d:]
        dd = np.abs(second[:, diag_idx])                     # [N, d]
        S[:, :d] = np.sqrt(np.abs(gs[:, None] * dd))
        p = 0
        for r in range(d):
            for c in range(r + 1):
                S[:, d + p] = np.sqrt(dd[:, r] * dd[:, c])
                p += 1
    s[base:base + N * K] = S.ravel()
    return s


def assert_stats_close(got, ref, N, K_or_fam, tol, what="", d=1):
    """K_or_fam: the family name (preferred) or, for table models, 0."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    fam = K_or_fam if isinstance(K_or_fam, str) else "table"
    s = natural_scale(ref, fam, N, d)
    lim = tol * np.maximum(np.abs(ref), s)
    bad = ~(np.abs(got - ref) <= lim)
    if bad.any():
        i = int(np.argmax(np.abs(got - ref) / np.maximum(lim, 1e-300)))
        raise AssertionError(f"{what}: {bad.sum()} statistics off; worst index {i}: got "
                             f"{got[i]!r} ref {ref[i]!r} scale {s[i]!r} (tol {tol})")


def assert_loglik_close(got, ref, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got)), f"{what}: finiteness differs"
    err = np.abs(got[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)
    assert err.size == 0 or err.max() <= tol, f"{what}: loglik rel err {err.max():.3e} > {tol}"
