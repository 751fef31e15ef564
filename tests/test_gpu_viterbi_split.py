"""Viterbi on sequences longer than one forward segment (1,024 steps), against
the oracle, through the C ABI.

The forward max-plus recursion of such a sequence runs in segments swept in
parallel: a first sweep of each segment from the all-zero score vector, a
second from the vector stored at the end of the previous segment (stopping
where the two agree within a quarter of the near-tie threshold), and an
in-order pass that re-runs the segments without an agreement.  On FP64 tables
the returned path equals the oracle's wherever no near-tie (< 1e-12) is met,
the path log-probability agrees to 1e-12 and the near-tie count matches; a
chain that never forgets its start (the identity transition matrix) takes
the re-run path; a path that becomes impossible, or a non-finite
observation, in a later segment is reported as in the unsplit recursion.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

import oracle
import workloads
from tests.test_gpu_viterbi import path_score, run_vit

pytestmark = pytest.mark.gpu

LENGTHS = [1, 1023, 1024, 1025, 2047, 2048, 2049, 3100, 5000]


@pytest.fixture(scope="module")
def h():
    import paper_2605_29208_amd as h
    return h


def check_against_oracle(m, logB, offs, path, lp, nt, what, exact_ties=True):
    for b in range(len(offs) - 1):
        sl = slice(offs[b], offs[b + 1])
        rp, rlp, rties = oracle.viterbi(m.log_pi, m.log_A, logB[sl])
        if not np.array_equal(path[sl], rp):
            assert rties > 0, f"{what}: sequence {b} differs without a near-tie"
        elif exact_ties:
            assert nt[b] == rties, (what, b, nt[b], rties)
        assert abs(path_score(m.log_pi, m.log_A, logB[sl], path[sl]) - rlp) <= 1e-12 * abs(rlp)
        assert abs(lp[b] - rlp) <= 1e-12 * abs(rlp), (what, b, lp[b], rlp)


@pytest.mark.parametrize("n", [1, 2, 3, 8, 16, 33, 40, 64])
def test_viterbi_segments_table_f64(h, n):
    rng = np.random.default_rng(760 + n)
    offs = np.concatenate([[0], np.cumsum(LENGTHS)])
    logB = rng.normal(-2.0, 1.5, (offs[-1], n))
    m = workloads.make_model("gaussian", n, 1, rng)
    dm = h.DeviceModel("table", n, n, m.log_pi, m.log_A, None)
    path, lp, nt = run_vit(h, dm, logB, offs, "f64", want_ties=True)
    check_against_oracle(m, logB, offs, path, lp, nt, f"table N={n}")


@pytest.mark.parametrize("fam,n", [("gaussian", 16), ("poisson", 64), ("student_t", 32)])
def test_viterbi_segments_device_emissions(h, fam, n):
    w = workloads.random_workload(fam, n, 1, [4000, 1500, 900, 2500], 770 + n)
    m = w.model
    dm = h.DeviceModel.from_model(m)
    path64, lp64, nt64 = run_vit(h, dm, w.obs, w.offsets, "f64", want_ties=True)
    path32, lp32 = run_vit(h, dm, w.obs, w.offsets, "f32")
    logB = np.concatenate([oracle.emission(fam, n, 1, m.theta, w.obs[w.offsets[b]:w.offsets[b + 1]])
                           for b in range(w.n_seq)])
    check_against_oracle(m, logB, w.offsets, path64, lp64, nt64, f"{fam} N={n} f64",
                         exact_ties=False)
    for b in range(w.n_seq):
        sl = slice(w.offsets[b], w.offsets[b + 1])
        _, rlp, _ = oracle.viterbi(m.log_pi, m.log_A, logB[sl])
        assert path_score(m.log_pi, m.log_A, logB[sl], path32[sl]) >= rlp - 1e-4 * abs(rlp)
        assert abs(lp32[b] - rlp) <= 1e-4 * abs(rlp)


def test_viterbi_identity_chain_reruns(h):
    """With A = I every state's score runs on its own, so two sweeps from
    different starts never agree: every segment after the first is re-run in
    order.  The best path stays in the state with the best total."""
    rng = np.random.default_rng(780)
    n = 12
    with np.errstate(divide="ignore"):
        log_A = np.log(np.eye(n))
    log_pi = np.log(np.full(n, 1.0 / n))
    m = workloads.Model("table", n, n, log_pi, log_A, np.zeros(0))
    offs = np.array([0, 4500, 6000])
    logB = rng.normal(-2.0, 1.0, (offs[-1], n))
    dm = h.DeviceModel("table", n, n, log_pi, log_A, None)
    for prec in ("f64", "f32"):
        path, lp, nt = run_vit(h, dm, logB, offs, prec, want_ties=True)
        for b in range(2):
            sl = slice(offs[b], offs[b + 1])
            rp, rlp, _ = oracle.viterbi(log_pi, log_A, logB[sl])
            np.testing.assert_array_equal(path[sl], rp)
            tol = 1e-12 if prec == "f64" else 1e-4
            assert abs(lp[b] - rlp) <= tol * abs(rlp), (prec, b, lp[b], rlp)


def test_viterbi_dead_and_invalid_in_later_segments(h):
    """An impossible step (every state -inf) in the third segment of one
    sequence and a NaN in the second segment of another: log-probability -inf
    and NaN, path -1, no near-ties; the other sequences are unaffected."""
    rng = np.random.default_rng(790)
    n = 10
    m = workloads.make_model("gaussian", n, 1, rng)
    lengths = [3500, 2600, 1800]
    offs = np.concatenate([[0], np.cumsum(lengths)])
    logB = rng.normal(-2.0, 1.5, (offs[-1], n))
    logB[offs[0] + 2400, :] = -np.inf
    logB[offs[1] + 1500, 3] = np.nan
    dm = h.DeviceModel("table", n, n, m.log_pi, m.log_A, None)
    path, lp, nt = run_vit(h, dm, logB, offs, "f64", want_ties=True)
    assert lp[0] == -np.inf and np.all(path[offs[0]:offs[1]] == -1) and nt[0] == 0
    assert np.isnan(lp[1]) and np.all(path[offs[1]:offs[2]] == -1) and nt[1] == 0
    sl = slice(offs[2], offs[3])
    rp, rlp, rties = oracle.viterbi(m.log_pi, m.log_A, logB[sl])
    np.testing.assert_array_equal(path[sl], rp)
    assert abs(lp[2] - rlp) <= 1e-12 * abs(rlp) and nt[2] == rties
