"""Sweep segments of the batched E-step for 8 < N <= 64 states, against the
FP64 oracle through the C ABI.

Long sequences are cut into segments swept in parallel: a first sweep of
every segment from a vector of ones, a second one from the vector its
neighbour stored (stopping where the two agree), and an in-order pass that
re-runs the segments whose second sweep found no agreement.  Every segment
length the schedule can take (1024, whole sequences, 512, 2048 steps) is
forced in turn on lengths at and around its multiples.  Chains that forget
their start slowly or never (uninformative emissions over long stretches, a
near-identity or identity transition matrix) take the re-run path; a path
that becomes impossible inside a later segment gives status 1; results do not
depend on the rest of the batch.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

import oracle
import workloads
from tests.parity import TOL, assert_loglik_close, assert_stats_close

pytestmark = pytest.mark.gpu

# around the multiples of 512, 1024 and 2048 steps, and a long tail
LENGTHS = [1, 31, 511, 512, 513, 1023, 1024, 1025, 1056, 2047, 2048, 2049, 3000, 4097, 6100]
VARIANTS = 4


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_29208_amd as h
    yield h
    h.hmm_set_variant(-1)


def estep(h, model, offsets, obs, prec, variant):
    import torch
    dm = h.DeviceModel("table", model.n_states, model.n_states, model.log_pi, model.log_A, None) \
        if model.family == "table" else h.DeviceModel.from_model(model)
    db = h.DeviceBatch(obs, offsets, dtype=np.float64 if prec == "f64" else np.float32)
    try:
        h.hmm_set_variant(variant)
        assert h.hmm_get_variant(dm, db, prec) == (variant, VARIANTS)
        stats, ll, st = h.estep_stats(dm, db, prec)
        torch.cuda.synchronize()
    finally:
        h.hmm_set_variant(-1)
    return stats.cpu().numpy(), ll.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("fam,n,precs", [("student_t", 32, ("f32", "f64")),
                                         ("gaussian", 16, ("f32", "f64")),
                                         ("poisson", 64, ("f32",)),
                                         ("gamma", 9, ("f32", "f64")),
                                         ("gaussian", 17, ("f64",)),
                                         ("student_t", 47, ("f32",))])
def test_segments_every_variant(h, fam, n, precs):
    w = workloads.random_workload(fam, n, 1, LENGTHS, 700 + n)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    for prec in precs:
        for v in range(VARIANTS):
            stats, ll, st = estep(h, w.model, w.offsets, w.obs, prec, v)
            what = f"{fam} N={n} {prec} variant {v}"
            assert np.array_equal(st, ref["status"]), what
            assert_loglik_close(ll, ref["loglik"], TOL[prec], what)
            assert_stats_close(stats, ref["stats"], n, fam, TOL[prec], what)


def table_model(rng, n, A):
    with np.errstate(divide="ignore"):
        return workloads.Model("table", n, n, np.log(np.full(n, 1.0 / n)), np.log(A), np.zeros(0))


def mixed_table(rng, n, T, quiet):
    """Log-emission rows: informative (Dirichlet rows over nine symbols)
    except on the steps in `quiet`, where every state has the same density."""
    logB = np.log(rng.dirichlet(np.ones(9), size=n).T[rng.integers(0, 9, T)])
    logB[quiet] = -1.0
    return logB


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_slow_forgetting_reruns(h, prec):
    """Uninformative stretches under a sticky chain (self-transition 0.995):
    there the chain forgets its start over thousands of steps, so second
    sweeps find no agreement and segments are re-run in order; elsewhere
    they agree.  The identity chain never forgets, so every segment of its
    sequence is re-run."""
    rng = np.random.default_rng(710)
    n = 24
    A = 0.995 * np.eye(n) + 0.005 * rng.dirichlet(np.ones(n), size=n)
    lengths = [6000, 3500, 700]
    T = sum(lengths)
    quiet = np.zeros(T, dtype=bool)
    quiet[1500:4200] = True
    quiet[6000 + 1100:6000 + 3300] = True
    logB = mixed_table(rng, n, T, quiet)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    m = table_model(rng, n, A)
    ref = oracle.estep(m, offs, None, logB=logB)
    for v in (0, 2):
        stats, ll, st = estep(h, m, offs, logB, prec, v)
        assert (st == 0).all()
        assert_loglik_close(ll, ref["loglik"], TOL[prec], f"sticky {prec} variant {v}")
        assert_stats_close(stats, ref["stats"], n, 0, TOL[prec], f"sticky {prec} variant {v}")
    # the identity chain: pi keeps its weights, each state's likelihood runs alone
    mi = table_model(rng, n, np.eye(n))
    lb = mixed_table(rng, n, 5000, np.arange(5000) % 3 == 0)
    offs1 = np.array([0, 5000])
    ref1 = oracle.estep(mi, offs1, None, logB=lb)
    stats, ll, st = estep(h, mi, offs1, lb, prec, 2)
    assert (st == 0).all()
    assert_loglik_close(ll, ref1["loglik"], TOL[prec], f"identity {prec}")
    assert_stats_close(stats, ref1["stats"], n, 0, TOL[prec], f"identity {prec}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_path_dies_in_a_later_segment(h, prec):
    """A chain that stays in its starting state, started in state 0, meets a
    step that state 0 cannot emit in its third segment: log-likelihood -inf
    and status 1, although every other state could go on.  The other
    sequences' statistics still match.  State 0 has the highest density at
    every other step, so the backward vectors keep it as their largest entry."""
    rng = np.random.default_rng(720)
    n = 12
    with np.errstate(divide="ignore"):
        log_pi = np.log(np.eye(n)[0])
        log_A = np.log(np.eye(n))
    m = workloads.Model("table", n, n, log_pi, log_A, np.zeros(0))
    lengths = [4000, 900, 2500]
    T = sum(lengths)
    logB = np.log(rng.dirichlet(np.ones(9), size=n).T[rng.integers(0, 9, T)])
    logB[:, 0] = logB.max(axis=1) + 0.1
    logB[2600, 0] = -np.inf
    offs = np.concatenate([[0], np.cumsum(lengths)])
    ref = oracle.estep(m, offs, None, logB=logB)
    assert list(ref["status"]) == [1, 0, 0]
    for v in (0, 2, 1):
        stats, ll, st = estep(h, m, offs, logB, prec, v)
        assert list(st) == [1, 0, 0], (prec, v, st)
        assert ll[0] == -np.inf
        assert_loglik_close(ll[1:], ref["loglik"][1:], TOL[prec], f"dead {prec} variant {v}")
        assert_stats_close(stats, ref["stats"], n, 0, TOL[prec], f"dead {prec} variant {v}")


def test_segments_batch_invariance_and_posteriors(h):
    import torch
    w = workloads.random_workload("student_t", 32, 1, [5000, 40, 2100, 1024, 3333], 730)
    _, ll, _ = estep(h, w.model, w.offsets, w.obs, "f32", 0)
    for k in (0, 2, 4):
        sub = w.subset([k])
        _, a, _ = estep(h, sub.model, sub.offsets, sub.obs, "f32", 0)
        assert a[0] == ll[k]
    # gamma of split sequences (default schedule) against the oracle, whose
    # own log-space rounding on 5,000-step sequences is about 1e-10, and
    # against the unsplit sweeps, which differ only where a second sweep
    # agreed (2^-40 or 2^-16 relative)
    ref = oracle.estep(w.model, w.offsets, w.obs, want_gamma=True)
    dm = h.DeviceModel.from_model(w.model)
    for prec, atol_ref, atol_split in (("f64", 2e-9, 1e-11), ("f32", 5e-5, 5e-5)):
        db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
        gams = []
        for v in (0, 1):
            try:
                h.hmm_set_variant(v)
                llg, gam, st = h.forward_backward(dm, db, prec)
                torch.cuda.synchronize()
            finally:
                h.hmm_set_variant(-1)
            assert (st.cpu().numpy() == 0).all()
            assert_loglik_close(llg.cpu().numpy(), ref["loglik"], TOL[prec], f"fb {prec} {v}")
            gams.append(gam.cpu().numpy().astype(np.float64))
        err = np.abs(gams[0] - ref["gamma"]).max()
        assert err <= atol_ref, (prec, err)
        diff = np.abs(gams[0] - gams[1]).max()
        assert diff <= atol_split, (prec, diff)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_segments_in_hip_graph_fresh_thread(h, prec):
    """The segmented E-step (three sweep launches) captured in a HIP graph
    from a host thread that never called the library before; every replay,
    with eager work and synchronisation between replays, equals the eager
    call bit for bit."""
    import threading
    import torch
    w = workloads.random_workload("student_t", 32, 1, [5000, 40, 2100, 1100], 740)
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
    S = h.hmm_stats_len(dm)
    stats = torch.zeros(S, dtype=torch.float64, device="cuda")
    ll = torch.empty(w.n_seq, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_seq, dtype=torch.int32, device="cuda")
    ws = h._ws(h.hmm_workspace_size("estep", dm, db, prec))
    h.hmm_estep_stats(dm, db, prec, stats, ll, st, ws)
    torch.cuda.synchronize()
    eager = (stats.clone(), ll.clone(), st.clone())
    assert (st.cpu().numpy() == 0).all()
    out = {}

    def capture_and_replay():
        try:
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=side):
                h.hmm_estep_stats(dm, db, prec, stats, ll, st, ws)
            for rep in range(3):
                stats.zero_()
                ll.zero_()
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                assert torch.equal(stats, eager[0]) and torch.equal(ll, eager[1]), rep
                assert torch.equal(st, eager[2]), rep
                _ = (stats * 2).sum().item()   # eager work between replays
            out["ok"] = True
        except BaseException as e:   # reported in the test's own thread
            out["err"] = e

    t = threading.Thread(target=capture_and_replay)
    t.start()
    t.join()
    if "err" in out:
        raise out["err"]
    assert out.get("ok")
