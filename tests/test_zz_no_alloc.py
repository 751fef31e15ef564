"""The allocation-free E-step (hmm_estep_stats_noalloc, static device
workspace) against hmm_estep_stats with a caller workspace, through the C
ABI: two calls in a row on each route (N <= 8 chunks, the wave path, the
large-state path), the second with a smaller batch, so the second call runs
over what the first left in the static area."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_29208_amd as h
    return h


def outputs(h, w, prec, noalloc):
    import torch
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
    S = h.hmm_stats_len(dm)
    stats = torch.full((S,), 7.0, dtype=torch.float64, device="cuda")
    ll = torch.full((w.n_seq,), 7.0, dtype=torch.float64, device="cuda")
    st = torch.full((w.n_seq,), 7, dtype=torch.int32, device="cuda")
    if noalloc:
        h.hmm_estep_stats_noalloc(dm, db, prec, stats, ll, st)
    else:
        ws = h._ws(h.hmm_workspace_size("estep", dm, db, prec))
        h.hmm_estep_stats(dm, db, prec, stats, ll, st, ws)
    torch.cuda.synchronize()
    return stats.cpu().numpy(), ll.cpu().numpy(), st.cpu().numpy()


CASES = [("gamma", 8, 1, [700, 31, 2048, 1, 999], [5, 300, 64]),
         ("student_t", 32, 1, [1500, 40, 3001], [33, 900]),
         ("diag", 100, 4, [400, 7, 650], [129, 2])]


@pytest.mark.parametrize("fam,n,d,big,small", CASES)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_workspace_call(h, fam, n, d, big, small, prec):
    for k, lengths in enumerate((big, small)):
        w = workloads.random_workload(fam, n, d, lengths, 900 + 10 * n + k)
        ref = outputs(h, w, prec, noalloc=False)
        got = outputs(h, w, prec, noalloc=True)
        assert (ref[2] == 0).all()
        # same kernels on the same inputs, fixed reduction order: identical bits
        assert np.array_equal(got[2], ref[2])
        assert np.array_equal(got[1], ref[1]), (fam, n, prec, k)
        assert np.array_equal(got[0], ref[0]), (fam, n, prec, k)


def test_noalloc_rejects_oversized_batch(h):
    """A batch whose workspace exceeds the static area is refused on the host
    before anything is enqueued."""
    w = workloads.random_workload("gaussian", 200, 1, [60000, 60000], 990)
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float32)
    need = h.hmm_workspace_size("estep", dm, db, "f32")
    assert need > (64 << 20)
    import torch
    S = h.hmm_stats_len(dm)
    stats = torch.zeros(S, dtype=torch.float64, device="cuda")
    with pytest.raises(h.HmmError) as ei:
        h.hmm_estep_stats_noalloc(dm, db, "f32", stats, None, None)
    assert ei.value.status == 3 and "static area" in str(ei.value)
