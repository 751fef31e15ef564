"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances: 1e-9 relative for the FP64 paths, 1e-4 relative for the FP32
paths (log-likelihoods and pooled statistics).  A statistic near zero is
compared against its block's scale: |got - ref| <= tol * max(|ref|, 1e-3 *
max|block|), so entries that cancel (shifted first moments) are judged
relative to the size of the quantities they are made of.
"""
import numpy as np

TOL = {"f64": 1e-9, "plain_f64": 1e-9, "f32": 1e-4, "plain_f32": 1e-4}


def stat_blocks(N, K):
    b = [("loglik", slice(0, 1)), ("gamma1", slice(1, 1 + N)),
         ("xi", slice(1 + N, 1 + N + N * N)), ("gamma_sum", slice(1 + N + N * N, 1 + 2 * N + N * N))]
    base = 1 + 2 * N + N * N
    for k in range(K):
        b.append((f"fam{k}", slice(base + k, base + N * K, K)))
    return b


def assert_stats_close(got, ref, N, K, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    for name, sl in stat_blocks(N, K):
        g, r = got[sl], ref[sl]
        floor = 1e-3 * np.max(np.abs(r)) if r.size else 0.0
        lim = tol * np.maximum(np.abs(r), floor)
        bad = ~(np.abs(g - r) <= lim)
        if bad.any():
            i = int(np.argmax(np.abs(g - r) / np.maximum(lim, 1e-300)))
            raise AssertionError(f"{what} stats block {name}: {bad.sum()} entries off; worst "
                                 f"idx {i}: got {g[i]!r} ref {r[i]!r} (tol {tol})")


def assert_loglik_close(got, ref, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got)), f"{what}: finiteness differs"
    err = np.abs(got[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)
    assert err.size == 0 or err.max() <= tol, f"{what}: loglik rel err {err.max():.3e} > {tol}"


def family_k(fam, d=1):
    return {"gaussian": 2, "gamma": 3, "student_t": 4, "poisson": 1, "diag": 2 * d,
            "full": d + d * (d + 1) // 2, "table": 0}[fam]
