"""GPU parity of the batched E-step for large state counts and for the
multivariate families (one workgroup per sequence, emission table, xi as a
GEMM over stored alpha and w') against the FP64 oracle, through the C ABI.

The large-state workload (256 sequences of 2048 steps, N = 256 diagonal
Gaussian states in D = 16) runs at full size in the benchmark's launch
configuration and is checked on a sampled sequence plus exact identities.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

import oracle
import workloads
from tests.oracle_pool import pooled_estep
from tests.parity import TOL, assert_loglik_close, assert_stats_close

pytestmark = pytest.mark.gpu

LENGTHS = [1, 2, 31, 64, 65, 200]


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_29208_amd as h
    return h


def run_estep(h, w, prec, model=None, obs=None):
    import torch
    m = model if model is not None else w.model
    dm = h.DeviceModel.from_model(m)
    dt = np.float64 if prec in ("f64", "plain_f64") else np.float32
    db = h.DeviceBatch(w.obs if obs is None else obs, w.offsets, dtype=dt)
    stats, ll, st = h.estep_stats(dm, db, prec)
    torch.cuda.synchronize()
    return stats.cpu().numpy(), ll.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("fam", ["gaussian", "gamma", "student_t", "poisson"])
@pytest.mark.parametrize("n", [65, 128, 150, 200, 256])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_block_scalar_families(h, fam, n, prec):
    w = workloads.random_workload(fam, n, 1, LENGTHS, 800 + n)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    stats, ll, st = run_estep(h, w, prec)
    assert np.array_equal(st, ref["status"])
    assert_loglik_close(ll, ref["loglik"], TOL[prec], f"{fam} N={n} {prec}")
    assert_stats_close(stats, ref["stats"], n, fam, TOL[prec], f"{fam} N={n} {prec}")


@pytest.mark.parametrize("n,d", [(3, 2), (20, 5), (70, 16), (256, 16), (5, 40)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_block_diag_family(h, n, d, prec):
    w = workloads.random_workload("diag", n, d, [1, 40, 130], 820 + n + d)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    stats, ll, st = run_estep(h, w, prec)
    assert np.array_equal(st, ref["status"])
    assert_loglik_close(ll, ref["loglik"], TOL[prec], f"diag N={n} D={d} {prec}")
    assert_stats_close(stats, ref["stats"], n, "diag", TOL[prec], f"diag N={n} D={d} {prec}", d=d)


@pytest.mark.parametrize("n,d", [(3, 2), (8, 5), (4, 17), (32, 32), (3, 40), (2, 64)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_block_full_family(h, n, d, prec):
    w = workloads.random_workload("full", n, d, [1, 40, 130], 830 + n + d)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    stats, ll, st = run_estep(h, w, prec)
    assert np.array_equal(st, ref["status"])
    assert_loglik_close(ll, ref["loglik"], TOL[prec], f"full N={n} D={d} {prec}")
    assert_stats_close(stats, ref["stats"], n, "full", TOL[prec], f"full N={n} D={d} {prec}", d=d)


def truncate(w, tmax):
    """The same sequences cut to their first tmax steps."""
    lens = np.minimum(w.lengths, tmax)
    rows = np.concatenate([np.arange(w.offsets[b], w.offsets[b] + lens[b]) for b in range(len(lens))])
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return workloads.Workload(w.name, w.model, lens, offs, w.obs[rows], w.states[rows])


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config4a_subset(h, prec):
    """Full covariance, D = 32, condition numbers up to 1e3.  log P(y) reaches
    ~1e5 here, and the oracle's unnormalised log-space recursion carries about
    u * sqrt(T) * |log P| of absolute rounding (u = 2^-53): ~1e-9 at T = 4000,
    the FP64 tolerance itself.  FP64 is therefore compared on the sequences cut
    to 600 steps; FP32 on the whole sequences."""
    w = workloads.config4a(n_seq=3)
    if prec == "f64":
        w = truncate(w, 600)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    stats, ll, st = run_estep(h, w, prec)
    assert (st == 0).all()
    assert_loglik_close(ll, ref["loglik"], TOL[prec], f"config4a subset {prec}")
    assert_stats_close(stats, ref["stats"], 32, "full", TOL[prec], f"config4a subset {prec}", d=32)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_block_table_family(h, prec):
    import torch
    n = 100
    rng = np.random.default_rng(840)
    lengths = [1, 40, 97]
    T = sum(lengths)
    logB = np.log(rng.dirichlet(np.ones(12), size=n).T[rng.integers(0, 12, T)])
    offs = np.concatenate([[0], np.cumsum(lengths)])
    base = workloads.make_model("gaussian", n, 1, rng)
    m = workloads.Model("table", n, n, base.log_pi, base.log_A, np.zeros(0))
    ref = oracle.estep(m, offs, None, logB=logB)
    dm = h.DeviceModel("table", n, n, m.log_pi, m.log_A, None)
    db = h.DeviceBatch(logB, offs, dtype=np.float64 if prec == "f64" else np.float32)
    stats, ll, st = h.estep_stats(dm, db, prec)
    torch.cuda.synchronize()
    assert_loglik_close(ll.cpu().numpy(), ref["loglik"], TOL[prec], "table")
    assert_stats_close(stats.cpu().numpy(), ref["stats"], n, 0, TOL[prec], "table")


@pytest.mark.parametrize("fam,n,d", [("full", 5, 3), ("diag", 7, 4), ("gaussian", 100, 1)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_block_posteriors_and_decode(h, fam, n, d, prec):
    import torch
    w = workloads.random_workload(fam, n, d, [1, 45, 160], 850 + n)
    ref = oracle.estep(w.model, w.offsets, w.obs, want_gamma=True)
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
    ll, gam, st = h.forward_backward(dm, db, prec)
    path, _ = h.posterior_decode(dm, db, prec)
    torch.cuda.synchronize()
    assert_loglik_close(ll.cpu().numpy(), ref["loglik"], TOL[prec], f"{fam} fb loglik")
    g = gam.cpu().numpy().astype(np.float64)
    atol = 1e-11 if prec == "f64" else 5e-5
    assert np.abs(g - ref["gamma"]).max() <= atol
    rp = oracle.posterior_decode(ref["gamma"])
    srt = np.sort(ref["gamma"], axis=1)
    gap = srt[:, -1] - srt[:, -2]
    assert np.all((path.cpu().numpy() == rp) | (gap < 1e-4))


def test_block_status_codes_and_exclusion(h):
    w = workloads.random_workload("gamma", 80, 1, [50, 60, 70, 33], 860)
    obs = w.obs.copy()
    obs[w.offsets[1] + 5] = np.nan          # non-finite observation -> status 2
    obs[w.offsets[2] + 40] = -1.0           # outside the Gamma support -> status 1
    ref = oracle.estep(w.model, w.offsets, obs)
    for prec in ("f32", "f64"):
        stats, ll, st = run_estep(h, w, prec, obs=obs)
        assert list(st) == list(ref["status"]) == [0, 2, 1, 0], (prec, st)
        assert ll[2] == -np.inf and np.isnan(ll[1])
        assert_stats_close(stats, ref["stats"], 80, "gamma", TOL[prec], f"status {prec}")


def test_block_determinism(h):
    w = workloads.random_workload("gaussian", 150, 1, [300, 1000, 77, 1], 870)
    a = run_estep(h, w, "f32")
    b = run_estep(h, w, "f32")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config3_subset(h, prec):
    w = workloads.config3(n_seq=3, T=300)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    stats, ll, st = run_estep(h, w, prec)
    assert (st == 0).all()
    assert_loglik_close(ll, ref["loglik"], TOL[prec], f"config3 subset {prec}")
    assert_stats_close(stats, ref["stats"], 256, "diag", TOL[prec], f"config3 subset {prec}", d=16)


def test_config3_full_size(h):
    """256 sequences of 2048 steps, N = 256, D = 16, as the benchmark launches
    them: a sampled sequence against the oracle, identities that hold at any
    size, and FP32 against FP64 on every pooled statistic."""
    w = workloads.config3()
    stats, ll, st = run_estep(h, w, "f32")
    assert (st == 0).all()
    B = len(w.offsets) - 1
    pick = np.array([37])
    sub = w.subset(pick)
    ref = oracle.estep(sub.model, sub.offsets, sub.obs)
    assert_loglik_close(ll[pick], ref["loglik"], TOL["f32"], "config3 sampled")
    N = 256
    g1 = stats[1:1 + N]
    xi = stats[1 + N:1 + N + N * N]
    gs = stats[1 + N + N * N:1 + 2 * N + N * N]
    total = int(w.offsets[-1])
    assert abs(g1.sum() - B) < 1e-4 * B
    assert abs(gs.sum() - total) < 1e-4 * total
    assert abs(xi.sum() - (total - B)) < 1e-4 * total
    assert abs(stats[0] - ll.sum()) < 1e-9 * abs(stats[0])
    s64, ll64, _ = run_estep(h, w, "f64")
    assert_loglik_close(ll, ll64, TOL["f32"], "config3 f32 vs f64")
    assert_stats_close(stats, s64, N, "diag", TOL["f32"], "config3 f32 vs f64", d=16)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config3_multi_slice(h, prec):
    """Nine sequences of 2048 steps (18,432 rows): the transition contraction
    runs over many row slices whose partials are summed in FP64, and the
    sweeps cross every prefetch window; every statistic against the oracle."""
    w = workloads.config3(n_seq=9, T=2048)
    ref = pooled_estep(w, groups=9)
    stats, ll, st = run_estep(h, w, prec)
    assert (st == 0).all() and (ref["status"] == 0).all()
    assert_loglik_close(ll, ref["loglik"], TOL[prec], f"config3 9x2048 {prec}")
    assert_stats_close(stats, ref["stats"], 256, "diag", TOL[prec], f"config3 9x2048 {prec}", d=16)


def _config4a_prefix(min_steps):
    """The first sequences of the full-covariance workload whose lengths add
    up to more than min_steps."""
    w = workloads.config4a()
    k = int(np.searchsorted(np.cumsum(w.lengths), min_steps)) + 1
    return w.subset(np.arange(k))


def test_config4a_multi_tile(h):
    """Full covariance, D = 32, FP32, on more than 2 x 8192 steps: the
    matrix-core family sums run several step tiles and merge them; every
    statistic against the oracle."""
    w = _config4a_prefix(2 * 8192 + 1)
    assert w.total_steps > 2 * 8192
    ref = pooled_estep(w)
    stats, ll, st = run_estep(h, w, "f32")
    assert (st == 0).all() and (ref["status"] == 0).all()
    assert_loglik_close(ll, ref["loglik"], TOL["f32"], "config4a multi-tile f32")
    assert_stats_close(stats, ref["stats"], 32, "full", TOL["f32"], "config4a multi-tile f32", d=32)


def test_config4a_full_size(h):
    """All 512 full-covariance sequences as the benchmark launches them:
    sampled sequences against the oracle, identities that hold at any size,
    and the FP32 path against the FP64 one."""
    w = workloads.config4a()
    stats, ll, st = run_estep(h, w, "f32")
    assert (st == 0).all()
    B = w.n_seq
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(B, 6, replace=False))
    sub = w.subset(pick)
    ref = pooled_estep(sub, groups=6)
    assert_loglik_close(ll[pick], ref["loglik"], TOL["f32"], "config4a sampled")
    N = 32
    g1 = stats[1:1 + N]
    xi = stats[1 + N:1 + N + N * N]
    gs = stats[1 + N + N * N:1 + 2 * N + N * N]
    total = w.total_steps
    assert abs(g1.sum() - B) < 1e-4 * B
    assert abs(gs.sum() - total) < 1e-4 * total
    assert abs(xi.sum() - (total - B)) < 1e-4 * total
    assert abs(stats[0] - ll.sum()) < 1e-9 * abs(stats[0])
    s64, ll64, _ = run_estep(h, w, "f64")
    assert_loglik_close(ll, ll64, TOL["f32"], "config4a f32 vs f64")
    assert_stats_close(stats, s64, N, "full", TOL["f32"], "config4a f32 vs f64", d=32)


@pytest.mark.parametrize("prec", ["f32", "f64", "bf16_scaled"])
def test_block_estep_in_hip_graph_fresh_thread(h, prec):
    """A large-state E-step captured in a HIP graph from a host thread that
    never called the library before: nothing in the call allocates or sets
    itself up lazily, and every replay (with eager work and synchronisation
    between replays) equals the eager call bit for bit."""
    import threading
    import torch
    w = workloads.random_workload("gaussian", 100, 1, [300, 1000, 77, 1, 500], 880)
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
