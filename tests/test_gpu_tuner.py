"""The E-step's schedule variants and the autotuner, through the C ABI.

Every variant the tuner can pick (chunk lengths 16/32/64 of the N <= 8
route, half/nominal/double slicing of the large-state transition
contraction, sweep segments of 1024 steps, whole sequences, 512 or 2048
steps for 8 < N <= 64) is forced in turn and compared with the FP64 oracle; the tuner
itself must return one of them, make later calls take it, and append its
choice to the file named by HMM_TUNE_CACHE."""
import os

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

import oracle
import workloads
from tests.parity import TOL, assert_loglik_close, assert_stats_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_29208_amd as h
    yield h
    h.hmm_set_variant(-1)


def run(h, w, prec):
    import torch
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
    stats, ll, st = h.estep_stats(dm, db, prec)
    torch.cuda.synchronize()
    return stats.cpu().numpy(), ll.cpu().numpy(), st.cpu().numpy(), dm, db


# lengths across chunk (16/32/64) and superchunk boundaries, and a long one
CASES = [("gamma", 8, 1, [1, 15, 16, 17, 63, 64, 65, 300, 1025, 4100], 1401),
         ("poisson", 3, 1, [2, 31, 33, 257, 700], 1402),
         ("gaussian", 150, 1, [1, 64, 200, 1900], 1403),
         ("diag", 100, 4, [1, 40, 700], 1404),
         ("gaussian", 256, 1, [3, 129, 1200], 1405),
         ("student_t", 32, 1, [1, 33, 600, 1025, 2100, 2600], 1406)]


@pytest.mark.parametrize("fam,n,d,lengths,seed", CASES)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_every_variant_matches_oracle(h, fam, n, d, lengths, seed, prec):
    w = workloads.random_workload(fam, n, d, lengths, seed)
    ref = oracle.estep(w.model, w.offsets, w.obs)
    try:
        h.hmm_set_variant(0)
        _, _, _, dm, db = run(h, w, prec)
        _, nv = h.hmm_get_variant(dm, db, prec)
        wave = 8 < n <= (32 if prec == "f64" else 64)
        assert nv == (4 if wave else (2 if (n <= 8 and prec == "f64") else 3))
        for v in range(nv):
            h.hmm_set_variant(v)
            stats, ll, st, dm, db = run(h, w, prec)
            assert h.hmm_get_variant(dm, db, prec) == (v, nv)
            assert (st == 0).all()
            assert_loglik_close(ll, ref["loglik"], TOL[prec], f"{fam} N={n} {prec} variant {v}")
            assert_stats_close(stats, ref["stats"], n, fam, TOL[prec],
                               f"{fam} N={n} {prec} variant {v}", d=d)
    finally:
        h.hmm_set_variant(-1)


@pytest.mark.parametrize("fam,n,d,lengths", [("gamma", 8, 1, [700, 1500, 64, 3000]),
                                             ("gaussian", 150, 1, [500, 1300, 2048])])
def test_autotune_picks_and_records(h, fam, n, d, lengths, tmp_path):
    import torch
    w = workloads.random_workload(fam, n, d, lengths, 1410 + n)
    cache = tmp_path / "tune.txt"
    os.environ["HMM_TUNE_CACHE"] = str(cache)
    try:
        h.hmm_set_variant(-1)
        dm = h.DeviceModel.from_model(w.model)
        db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float32)
        ws = h._ws(h.hmm_workspace_size("estep", dm, db, "f32"))
        S = h.hmm_stats_len(dm)
        stats = torch.empty(S, dtype=torch.float64, device="cuda")
        ll = torch.empty(w.n_seq, dtype=torch.float64, device="cuda")
        st = torch.empty(w.n_seq, dtype=torch.int32, device="cuda")
        v, ms = h.hmm_autotune(dm, db, "f32", stats, ll, st, ws)
        assert len(ms) == 3 and 0 <= v < 3
        assert all(t > 0 for t in ms) and ms[v] == min(ms)
        # later calls with this key take the chosen variant
        assert h.hmm_get_variant(dm, db, "f32") == (v, 3)
        line = cache.read_text().strip().splitlines()[-1].split()
        assert line[0].endswith(f"|N{n}|D{d}|prec1|route{1 if n <= 8 else 3}|B2|Tmean{int(np.ceil(np.log2(w.total_steps / w.n_seq)))}|Tmax{int(np.ceil(np.log2(max(lengths))))}")
        assert int(line[1]) == v
        # the tuned call still matches the oracle
        h.hmm_estep_stats(dm, db, "f32", stats, ll, st, ws)
        torch.cuda.synchronize()
        ref = oracle.estep(w.model, w.offsets, w.obs)
        assert_stats_close(stats.cpu().numpy(), ref["stats"], n, fam, TOL["f32"], "tuned")
    finally:
        os.environ.pop("HMM_TUNE_CACHE", None)
