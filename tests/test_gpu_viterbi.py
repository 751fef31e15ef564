"""GPU Viterbi (section 3.3) against the oracle.

FP64 on caller-supplied log-emission tables must reproduce the oracle bit
for bit (same operations in the same order).  With emissions evaluated on
the device (ocml vs glibc may differ in the last bit) paths may differ only
where the oracle reports a near-tie (< 1e-12); the log-probability of the
returned path is then optimal to 1e-12.  FP32 paths are checked for
optimality of their FP64-evaluated score to 1e-4 (relative), and the
mismatch rate against the FP64 path is reported.  The device's near-tie
count (n_ties) equals the oracle's on FP64 tables, where the candidate scores
are bitwise identical.
"""
import numpy as np
import pytest
import torch  # noqa: F401

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2605_29208_amd as h
    return h


def path_score(log_pi, log_A, logB, path):
    s = log_pi[path[0]] + logB[0, path[0]]
    if len(path) > 1:
        s += np.sum(log_A[path[:-1], path[1:]]) + np.sum(logB[np.arange(1, len(path)), path[1:]])
    return float(s)


def run_vit(h, dm, obs, offs, prec, want_ties=False):
    dt = np.float64 if prec == "f64" else np.float32
    db = h.DeviceBatch(obs, offs, dtype=dt)
    path, lp, ties = h.viterbi(dm, db, prec)
    torch.cuda.synchronize()
    if want_ties:
        return path.cpu().numpy(), lp.cpu().numpy(), ties.cpu().numpy()
    return path.cpu().numpy(), lp.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 33, 64])
def test_viterbi_table_f64_bit_exact(h, n):
    rng = np.random.default_rng(600 + n)
    lengths = [1, 2, 63, 64, 65, 200, 333]
    offs = np.concatenate([[0], np.cumsum(lengths)])
    logB = rng.normal(-2.0, 1.5, (offs[-1], n))
    m = workloads.make_model("gaussian", n, 1, rng)
    dm = h.DeviceModel("table", n, n, m.log_pi, m.log_A, None)
    path, lp, nt = run_vit(h, dm, logB, offs, "f64", want_ties=True)
    for b in range(len(lengths)):
        sl = slice(offs[b], offs[b + 1])
        rp, rlp, rties = oracle.viterbi(m.log_pi, m.log_A, logB[sl])
        np.testing.assert_array_equal(path[sl], rp)
        assert lp[b] == rlp
        assert nt[b] == rties


def test_viterbi_tie_rule_and_dead_sequence(h):
    n = 3
    log_pi = np.log(np.full(n, 1 / 3))
    log_A = np.log(np.full((n, n), 1 / 3))
    lengths = [5, 70]
    offs = np.array([0, 5, 75])
    logB = np.zeros((75, n))
    logB[5 + 10, :] = -np.inf          # second sequence: an impossible step
    dm = h.DeviceModel("table", n, n, log_pi, log_A, None)
    path, lp, nt = run_vit(h, dm, logB, offs, "f64", want_ties=True)
    assert list(path[:5]) == [0] * 5                      # exact ties -> lowest index
    assert abs(lp[0] - 5 * np.log(1 / 3)) < 1e-12
    assert lp[1] == -np.inf and np.all(path[5:] == -1)
    # every decision of the first sequence is an exact tie: the final state and
    # the four backpointers taken; the dead sequence reports none
    _, _, rties = oracle.viterbi(log_pi, log_A, logB[:5])
    assert rties == 5 and nt[0] == 5 and nt[1] == 0


def test_viterbi_near_tie_count_constructed(h):
    """Two states whose candidate scores differ by 1e-14 (a near-tie) at chosen
    steps and by 1e-6 elsewhere: the count along the path matches the oracle."""
    n = 2
    T = 40
    log_pi = np.log(np.array([0.5, 0.5]))
    log_A = np.log(np.array([[0.5, 0.5], [0.5, 0.5]]))
    logB = np.zeros((T, n))
    logB[:, 1] = -1e-6
    for t in (3, 17, 18, 31):
        logB[t, 1] = -1e-14
    dm = h.DeviceModel("table", n, n, log_pi, log_A, None)
    offs = np.array([0, T])
    path, lp, nt = run_vit(h, dm, logB, offs, "f64", want_ties=True)
    rp, rlp, rties = oracle.viterbi(log_pi, log_A, logB)
    np.testing.assert_array_equal(path, rp)
    assert lp[0] == rlp and nt[0] == rties and rties > 0


@pytest.mark.parametrize("fam,n", [("gaussian", 3), ("gamma", 8), ("student_t", 5),
                                   ("poisson", 4), ("gaussian", 20)])
def test_viterbi_device_emissions(h, fam, n):
    w = workloads.random_workload(fam, n, 1, [1, 64, 65, 500, 1000], 700 + n)
    m = w.model
    dm = h.DeviceModel.from_model(m)
    path64, lp64, nt64 = run_vit(h, dm, w.obs, w.offsets, "f64", want_ties=True)
    path32, lp32 = run_vit(h, dm, w.obs, w.offsets, "f32")
    mism = 0
    for b in range(w.n_seq):
        sl = slice(w.offsets[b], w.offsets[b + 1])
        logB = oracle.emission(fam, n, 1, m.theta, w.obs[sl])
        rp, rlp, ties = oracle.viterbi(m.log_pi, m.log_A, logB)
        if not np.array_equal(path64[sl], rp):
            assert ties > 0, f"sequence {b}: FP64 path differs without a near-tie"
        else:
            # same path: the device counts the same near-ties up to decisions
            # whose gap straddles the threshold by a rounding difference
            assert abs(int(nt64[b]) - ties) <= max(1, ties)
        assert abs(path_score(m.log_pi, m.log_A, logB, path64[sl]) - rlp) <= 1e-12 * abs(rlp)
        assert abs(lp64[b] - rlp) <= 1e-12 * abs(rlp)
        s32 = path_score(m.log_pi, m.log_A, logB, path32[sl])
        assert s32 >= rlp - 1e-4 * abs(rlp)
        assert abs(lp32[b] - rlp) <= 1e-4 * abs(rlp)
        mism += int(np.sum(path32[sl] != rp))
    print(f"{fam} N={n}: FP32 path mismatch rate {mism / w.total_steps:.2e}")


def test_viterbi_config1(h):
    w = workloads.config1()
    m = w.model
    dm = h.DeviceModel.from_model(m)
    path, lp = run_vit(h, dm, w.obs, w.offsets, "f64")
    logB = oracle.emission("gaussian", 3, 1, m.theta, w.obs)
    rp, rlp, ties = oracle.viterbi(m.log_pi, m.log_A, logB)
    assert np.array_equal(path, rp) or ties > 0
    assert abs(lp[0] - rlp) <= 1e-12 * abs(rlp)
    # the decoded path recovers most of the simulated hidden states
    assert np.mean(path == w.states) > 0.8
