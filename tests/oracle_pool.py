"""The FP64 oracle over a large batch, one group of sequences per host thread.

The pooled statistics are sums over sequences (reading R3), so the oracle's
per-group results are added in group order; log-likelihoods and statuses are
concatenated.  Test infrastructure only.
"""
import concurrent.futures as cf
import os

import numpy as np

import oracle


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def pooled_estep(w, groups=None):
    """oracle.estep over workload w, split into `groups` runs of consecutive sequences."""
    B = w.n_seq
    groups = groups or min(B, 4 * host_threads())
    bounds = np.linspace(0, B, groups + 1).astype(int)
    parts = [w.subset(np.arange(bounds[g], bounds[g + 1])) for g in range(groups)
             if bounds[g + 1] > bounds[g]]
    oracle._load()
    with cf.ThreadPoolExecutor(max_workers=host_threads()) as ex:
        res = list(ex.map(lambda p: oracle.estep(p.model, p.offsets, p.obs), parts))
    stats = np.zeros_like(res[0]["stats"])
    for r in res:
        stats += r["stats"]
    return {"stats": stats, "loglik": np.concatenate([r["loglik"] for r in res]),
            "status": np.concatenate([r["status"] for r in res])}
