"""Device M-steps (section 4) and the EM loop, against the FP64 oracle.

M-step parity: identical pooled statistics (computed by the oracle) go to
both sides; parameters agree to 1e-10 relative, collapse flags and Newton
iteration counts match.  One full EM iteration on the GPU (FP64 E-step +
M-steps) agrees with the oracle's iteration to 1e-9.  The EM loop captured
in a HIP graph replays identically to the eager loop, replay after replay.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2605_29208_amd as h
    return h


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


FAMS = [("gaussian", 3, 1), ("gamma", 5, 1), ("student_t", 4, 1), ("poisson", 4, 1),
        ("diag", 3, 4), ("full", 3, 5)]


@pytest.mark.parametrize("fam,n,d", FAMS)
def test_mstep_matches_oracle(h, fam, n, d):
    w = workloads.random_workload(fam, n, d, [300, 200, 400], 800 + n)
    m = workloads.perturb(w.model, np.random.default_rng(1))
    r = oracle.estep(m, w.offsets, w.obs)
    ref, rcol, rit = oracle.mstep_emission(fam, n, d, m.theta, r["stats"])
    dm = h.DeviceModel.from_model(m)
    st = dev(r["stats"])
    out = torch.empty_like(dm.theta)
    col = torch.empty(n, dtype=torch.int32, device="cuda")
    its = torch.empty(n, dtype=torch.int32, device="cuda")
    h.hmm_mstep(dm, st, h.default_mstep_opts(), out, col, its)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)
    assert np.array_equal(col.cpu().numpy(), rcol)
    if fam in ("gamma", "student_t"):
        assert np.abs(its.cpu().numpy() - rit).max() <= 1
    lp, la, _ = oracle.mstep_transitions(n, r["stats"], m.log_A)
    lpo, lao = torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty_like(dm.log_A)
    h.hmm_mstep_transitions(dm, st, None, lpo, lao)
    torch.cuda.synchronize()
    np.testing.assert_allclose(lpo.cpu().numpy(), lp, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(lao.cpu().numpy(), la, rtol=1e-12, atol=1e-14)


def test_collapse_guard_and_in_place(h):
    """A state with no occupancy keeps its parameters; a row with no
    transitions keeps its row; in-place and out-of-place give the same."""
    w = workloads.random_workload("gaussian", 3, 1, [50, 60], 850)
    m = w.model
    r = oracle.estep(m, w.offsets, w.obs)
    stats = r["stats"].copy()
    n = 3
    gs = 1 + n + n * n
    stats[gs + 2] = 0.0                           # state 2 never occupied
    stats[1 + n + 2 * n:1 + n + 3 * n] = 0.0      # no transitions out of state 2
    ref, rcol, _ = oracle.mstep_emission("gaussian", n, 1, m.theta, stats)
    _, la, kept = oracle.mstep_transitions(n, stats, m.log_A)
    assert rcol[2] == 1 and kept[2] == 1
    dm = h.DeviceModel.from_model(m)
    st = dev(stats)
    out = torch.empty_like(dm.theta)
    col = torch.empty(n, dtype=torch.int32, device="cuda")
    h.hmm_mstep(dm, st, None, out, col)
    h.hmm_mstep(dm, st, None, dm.theta, None)      # in place
    h.hmm_mstep_transitions(dm, st, None, dm.log_pi, dm.log_A)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-12)
    assert np.array_equal(out.cpu().numpy(), dm.theta.cpu().numpy())
    assert list(col.cpu().numpy()) == list(rcol)
    np.testing.assert_allclose(dm.log_A.cpu().numpy(), la, rtol=1e-12)


@pytest.mark.parametrize("fam,n", [("gamma", 8), ("student_t", 4)])
def test_em_iteration_matches_oracle(h, fam, n):
    w = workloads.random_workload(fam, n, 1, [700, 1500, 333, 2000], 860 + n)
    m0 = workloads.perturb(w.model, np.random.default_rng(2))
    ref, _ = oracle.em_iteration(m0, w.offsets, w.obs)
    dm = h.DeviceModel.from_model(m0)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64)
    S = h.hmm_stats_len(dm)
    stats = torch.empty(S, dtype=torch.float64, device="cuda")
    ll = torch.empty(w.n_seq, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_seq, dtype=torch.int32, device="cuda")
    ws = h._ws(h.hmm_workspace_size("estep", dm, db, "f64"))
    h.em_iteration(dm, db, "f64", stats, ll, st, ws)
    torch.cuda.synchronize()
    np.testing.assert_allclose(dm.theta.cpu().numpy(), ref.theta, rtol=1e-9)
    np.testing.assert_allclose(dm.log_A.cpu().numpy(), ref.log_A, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(dm.log_pi.cpu().numpy(), ref.log_pi, rtol=1e-9, atol=1e-12)


def test_em_loop_in_hip_graph(h):
    """K EM iterations (E-step + M-steps) captured once and replayed: every
    replay from the same start equals the eager loop bit for bit, with eager
    work and synchronisation between replays; the log-likelihood rises."""
    K = 5
    w = workloads.config2(n_seq=64)
    m0 = workloads.perturb(w.model, np.random.default_rng(3))
    dm = h.DeviceModel.from_model(m0)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float32)
    S = h.hmm_stats_len(dm)
    stats = torch.zeros((K, S), dtype=torch.float64, device="cuda")
    ll = torch.empty(w.n_seq, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_seq, dtype=torch.int32, device="cuda")
    ws = h._ws(h.hmm_workspace_size("estep", dm, db, "f32"))
    start = [t.clone() for t in (dm.log_pi, dm.log_A, dm.theta)]

    def reset():
        for dst, src in zip((dm.log_pi, dm.log_A, dm.theta), start):
            dst.copy_(src)

    def loop():
        for k in range(K):
            h.em_iteration(dm, db, "f32", stats[k], ll, st, ws)

    reset()
    loop()
    torch.cuda.synchronize()
    eager = (stats.clone(), dm.theta.clone(), dm.log_A.clone())
    traj = eager[0][:, 0].cpu().numpy()
    assert np.all(np.diff(traj) >= -1e-6 * np.abs(traj[1:])), traj

    g = torch.cuda.CUDAGraph()
    reset()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        loop()                      # warm-up on the capture stream's side
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        loop()
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        stats.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(stats, eager[0]), rep
        assert torch.equal(dm.theta, eager[1]) and torch.equal(dm.log_A, eager[2]), rep
        _ = (dm.theta * 2).sum().item()   # eager work between replays
