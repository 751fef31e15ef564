"""Benchmark: one Baum-Welch E-step over a batch of ragged sequences.

Default workload (--workload batched): 1024 sequences with lengths uniform in
{500..5000}, N = 8 Gamma states (shape U[1,10], scale U[0.5,3]), sticky A
(a_ii = 0.95).  --workload heavy: 512 sequences with log-normal lengths
(median 3000, sigma 0.6, at most 20,000), N = 32 Student-t states.
--workload large: 256 sequences of 2048 steps, N = 256 diagonal Gaussian
states in D = 16.  --workload full: the heavy workload's lengths with N = 32
full-covariance Gaussian states in D = 32.  FP32 observations resident in
device memory.  One step = one full E-step
(parameter staging, emission log-densities, forward and backward
recursions, posteriors and the pooled sufficient statistics).

Prints one JSON line with the throughput in state transitions per second
(sum_b T_b * N^2 per E-step), the plain one-thread-per-sequence GPU method
on the same data, the dominant kernel's roofline figures and the FP64 CPU
oracle timed on the host.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# the serving run keeps up to SERVING_STREAMS latency-bound launches in
# flight; HIP gives each stream its own hardware queue only up to this count
# (read once, when the HIP runtime starts)
SERVING_STREAMS = 16
os.environ.setdefault("GPU_MAX_HW_QUEUES", str(SERVING_STREAMS))

PEAK_FP32_VALU_TFLOPS = 157.3   # MI355X FP32 vector, spec sheet
PEAK_FP64_VALU_TFLOPS = 78.6    # MI355X FP64 vector
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense bf16 / fp16 matrix
METRIC = "E-step state-transitions/s (B*T*N^2) vs plain GPU; p50/p99 decode latency"


def log(msg):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(records, steps):
    agg = {}
    for name, ms in records:
        a = agg.setdefault(name, [0.0, 0])
        a[0] += ms
        a[1] += 1
    return {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / v[1],
                "ms_per_step": v[0] / steps} for k, v in agg.items()}


def algorithmic_flops(name, w):
    """FLOPs of the method's arithmetic for one launch of kernel `name`."""
    n = w.model.n_states
    steps = w.total_steps
    if name == "chunk_stats":
        # forward alpha*A, backward A*w and the xi outer product: 3 FMA per transition
        return 6.0 * steps * n * n
    if name == "chunk_product":
        # chunk transfer matrices: N^3 FMA per step after each sequence's first
        return 2.0 * (steps - w.n_seq) * n ** 3
    if name == "wave_stats":
        # chunk forward alpha*A, backward A*w and the xi outer product
        return 6.0 * steps * n * n
    if name == "wave_sweep":
        # forward alpha*A and backward A*w over every sequence
        return 4.0 * steps * n * n
    if name in ("block_fwd", "block_bwd"):
        # one vector-matrix product per step
        return 2.0 * steps * n * n
    if name == "block_xi":
        return 2.0 * (steps - 1) * n * n
    return None


WORKLOADS = {
    "batched": ("batched ragged E-step: B=1024, T~U{500..5000}, N=8 Gamma, FP32 obs",
                lambda workloads: workloads.config2()),
    "heavy": ("heavy-tailed E-step: B=512, T~lognormal(median 3000, sigma 0.6, <=20000), "
              "N=32 Student-t, FP32 obs", lambda workloads: workloads.config4b()),
    "large": ("large-state E-step: B=256, T=2048, N=256 diagonal Gaussian D=16, FP32 obs",
              lambda workloads: workloads.config3()),
    "full": ("full-covariance E-step: B=512, T~lognormal(median 3000, sigma 0.6, <=20000), "
             "N=32 full-covariance Gaussian D=32, FP32 obs", lambda workloads: workloads.config4a()),
}


# kernel -> source file; the committed counter summary records the source's
# SHA-256 next to the measured bytes, and the figure is used only while the
# source is unchanged
KERNEL_SOURCE = {"chunk_stats": "k_chunk.hip", "chunk_product": "k_chunk.hip",
                 "wave_stats": "k_wave.hip", "wave_sweep": "k_wave.hip",
                 "block_fwd": "k_block.hip", "block_bwd": "k_block.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.md")


def source_sha(kernel):
    import hashlib
    f = KERNEL_SOURCE.get(kernel)
    if f is None:
        return None
    with open(os.path.join(ROOT, "paper_2605_29208_amd", "csrc", f), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch (fetch + write) from the committed summary, or None."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    sha = source_sha(kernel)
    for ln in lines:
        if ln.startswith("traffic:"):
            f = dict(kv.split("=", 1) for kv in ln[len("traffic:"):].split())
            if f.get("kernel") == kernel and f.get("workload") == workload and f.get("sha") == sha:
                return float(f["fetch_bytes"]) + float(f["write_bytes"])
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, reps=2):
    import oracle
    oracle._load()
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.estep(w.model, w.offsets, w.obs)
    dt = time.perf_counter() - t0
    return {"value": reps * w.transitions / dt, "unit": "transitions/s", "cores": 1,
            "kind": "oracle",
            "sample": f"full workload ({w.n_seq} sequences, {w.total_steps} steps) x{reps}, "
                      f"FP64 oracle, 1 thread on {cpu_model()}, {dt:.1f} s"}


def estep_time(h, w, prec, steps):
    """Mean milliseconds of one E-step (events around `steps` calls) and the
    per-kernel table."""
    import torch
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if prec == "f64" else np.float32)
    ws = h._ws(h.hmm_workspace_size("estep", dm, db, prec))
    S = h.hmm_stats_len(dm)
    stats = torch.empty(S, dtype=torch.float64, device="cuda")
    ll = torch.empty(w.n_seq, dtype=torch.float64, device="cuda")
    st = torch.empty(w.n_seq, dtype=torch.int32, device="cuda")
    h.hmm_estep_stats(dm, db, prec, stats, ll, st, ws)
    torch.cuda.synchronize()
    h.hmm_profile_reset()
    h.hmm_profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        h.hmm_estep_stats(dm, db, prec, stats, ll, st, ws)
    e1.record()
    torch.cuda.synchronize()
    recs = h.hmm_profile_records()
    h.hmm_profile_enable(False)
    h.hmm_profile_reset()
    ok = bool((st.cpu().numpy() == 0).all())
    return e0.elapsed_time(e1) / steps, kernel_table(recs, steps), ok


def other_workloads(h, workloads, steps):
    """The other configurations' E-steps at full size (context for the
    headline line): heavy-tailed N = 32 Student-t, large-state N = 256
    diagonal Gaussian in FP32 and in the scaled bf16 / fp16 forms, and
    full-covariance N = 32, D = 32."""
    res = {}
    for key, make, precs in (("heavy_student_t_n32", workloads.config4b, ("f32",)),
                             ("large_diag_n256", workloads.config3, ("f32", "bf16_scaled", "f16_scaled")),
                             ("full_cov_n32_d32", workloads.config4a, ("f32",))):
        w = make()
        for prec in precs:
            ms, kt, ok = estep_time(h, w, prec, steps)
            res[f"{key}_{prec}"] = {
                "sequences": w.n_seq, "total_steps": w.total_steps, "n_states": w.model.n_states,
                "ms_per_estep": ms, "transitions_per_s": w.transitions / (ms / 1e3),
                "all_status_ok": ok,
                "kernels_ms": {k: round(v["ms_avg"], 4) for k, v in kt.items()}}
            log(f"{key} {prec}: {ms:.3f} ms per E-step")
        del w
    return res


def serving_bench(h, workloads, qps_list, seconds, pool_size=256, streams=SERVING_STREAMS):
    """Decode requests (half Viterbi, half posterior decoding) arriving as a
    Poisson process at each rate in qps_list against 16 resident models
    (N in {4, 16, 64}, Gaussian and Poisson emissions), lengths log-normal
    (median 2000, sigma 1.0, 16..100,000).  Latency = scheduled arrival ->
    path in host memory; throughput in sequence steps per second."""
    models = workloads.serving_models()
    rng = np.random.default_rng(5007)
    srv = h.Server(hbm_budget=16 << 30, host_staging=1 << 30, max_batch=64, n_streams=streams)
    try:
        ids = [srv.add_model(h.DeviceModel.from_model(m)) for m in models]
        lengths = workloads.serving_request_lengths(rng, pool_size)
        pool = []
        for i in range(pool_size):
            k = int(rng.integers(len(models)))
            w = workloads.simulate("serve", models[k], [int(lengths[i])], rng)
            kind = "viterbi" if rng.random() < 0.5 else "posterior_decode"
            pool.append((k, kind, np.ascontiguousarray(w.obs, dtype=np.float32)))
        # warm-up: every (model, kind) once
        warm = 0
        for k in range(len(models)):
            for kind in ("viterbi", "posterior_decode"):
                srv.submit(ids[k], kind, pool[0][2][:64])
                warm += 1
        while warm > 0:
            warm -= len(srv.poll(256, 100000))
        points = []
        for qps in qps_list:
            n_req = max(1, int(qps * seconds))
            arrivals = np.cumsum(rng.exponential(1.0 / qps, n_req))
            t0 = h.hmm_server_now() + 0.02
            sent = []

            def submitter():
                for i in range(n_req):
                    ta = t0 + arrivals[i]
                    while True:
                        d = ta - h.hmm_server_now()
                        if d <= 0:
                            break
                        if d > 2e-3:
                            time.sleep(d - 1e-3)
                    k, kind, obs = pool[i % pool_size]
                    sent.append((srv.submit(ids[k], kind, obs), ta, len(obs)))

            th = threading.Thread(target=submitter)
            th.start()
            done = {}
            while len(done) < n_req:
                for c in srv.poll(1024, 2000):
                    done[c["id"]] = c
            th.join()
            lat = np.array([done[r]["t_done"] - ta for r, ta, _ in sent])
            wait = np.array([done[r]["t_launch"] - ta for r, ta, _ in sent])
            serv = np.array([done[r]["t_done"] - done[r]["t_launch"] for r, _, _ in sent])
            bs = np.array([done[r]["batch_size"] for r, _, _ in sent])
            steps = sum(T for _, _, T in sent)
            span = max(done[r]["t_done"] for r, _, _ in sent) - t0
            bad = sum(1 for r, _, _ in sent if done[r]["status"] != 0)
            log(f"serving {qps:g} QPS done")
            points.append({"qps_offered": qps, "requests": n_req,
                           "qps_served": n_req / span, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                           "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                           "max_ms": 1e3 * float(lat.max()),
                           "queue_p50_ms": 1e3 * float(np.percentile(wait, 50)),
                           "service_p50_ms": 1e3 * float(np.percentile(serv, 50)),
                           "service_p99_ms": 1e3 * float(np.percentile(serv, 99)),
                           "seq_steps_per_s": steps / span, "mean_batch": float(bs.mean()),
                           "failed": bad})
        info = srv.info()
    finally:
        srv.close()
    return {"models": "16 resident: 6 x N=4, 5 x N=16, 5 x N=64, Gaussian/Poisson alternating",
            "lengths": "log-normal median 2000, sigma 1.0, clipped 16..100000",
            "mix": "50% Viterbi, 50% posterior decode, FP32", "seconds_per_point": seconds,
            "points": points, "launches": info["launches"], "pool_peak_bytes": info["pool_peak"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64", "bf16_scaled", "f16_scaled"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--chunk", type=int, default=0, help="chunk length (0 = library default)")
    ap.add_argument("--em-iters", type=int, default=20,
                    help="EM iterations captured in one HIP graph (0 = skip)")
    ap.add_argument("--serving-seconds", type=float, default=3.0,
                    help="seconds of Poisson arrivals per serving rate (0 = skip)")
    ap.add_argument("--serving-qps", default="100,1000,3000",
                    help="comma-separated request rates of the serving run")
    ap.add_argument("--serving-streams", type=int, default=SERVING_STREAMS,
                    help="launches the server keeps in flight")
    ap.add_argument("--eager-only", action="store_true",
                    help="time eager calls only (no HIP graph capture), e.g. under counters")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 256 MiB device copy (reference for traffic counters)")
    ap.add_argument("--others", type=int, default=3,
                    help="E-steps timed on each secondary workload (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding of the "
                                   "sequence batch is described but not built"}))
        sys.exit(2)

    import torch
    import paper_2605_29208_amd as h
    import workloads

    h.hmm_set_chunk_len(args.chunk)
    wl_name, wl_make = WORKLOADS[args.workload]
    w = wl_make(workloads)
    dm = h.DeviceModel.from_model(w.model)
    db = h.DeviceBatch(w.obs, w.offsets, dtype=np.float64 if args.prec == "f64" else np.float32)
    prec = args.prec
    ws = h._ws(h.hmm_workspace_size("estep", dm, db, prec))
    S = h.hmm_stats_len(dm)
    stats = torch.empty(S, dtype=torch.float64, device="cuda")
    loglik = torch.empty(w.n_seq, dtype=torch.float64, device="cuda")
    status = torch.empty(w.n_seq, dtype=torch.int32, device="cuda")

    def step(p=prec, wsp=ws):
        h.hmm_estep_stats(dm, db, p, stats, loglik, status, wsp)

    log(f"workload {args.workload}: {w.n_seq} sequences, {w.total_steps} steps, N={w.model.n_states}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warm-up done")
    # (1) eager calls with per-kernel hipEvents (the kernel table and roofline)
    h.hmm_profile_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    eager_ms = ev0.elapsed_time(ev1) / args.steps
    recs = h.hmm_profile_records()
    h.hmm_profile_enable(False)
    kt = kernel_table(recs, args.steps)
    assert (status.cpu().numpy() == 0).all()
    log(f"eager: {eager_ms:.3f} ms per E-step")
    # (2) the same E-steps captured once in a HIP graph and replayed (the way an
    # EM loop issues them): the timed value
    if args.eager_only:
        ms = eager_ms
    else:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g_est = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_est):
            for _ in range(args.steps):
                step()
        g_est.replay()
        torch.cuda.synchronize()
        ev0.record()
        g_est.replay()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        del g_est
        assert (status.cpu().numpy() == 0).all()
    log(f"graph replay: {ms:.3f} ms per E-step")

    # plain GPU method (one thread per sequence, literal log-sum-exp) on the same
    # data.  Its sequences run side by side (one thread each), so its time is
    # linear in the longest sequence; for large N it is timed on the same
    # batch cut to its first plain_t steps and scaled by T / plain_t.
    plain_ms, plain_note = None, None
    if args.plain_steps > 0:
        pprec = "plain_f64" if prec == "f64" else "plain_f32"
        scale = 1.0
        T_max = int(np.max(w.lengths))
        plain_t = max(16, int(2e8 // (w.model.n_states ** 2 * 64)))
        if T_max > plain_t:
            cut = np.minimum(w.lengths, plain_t)
            offs = np.concatenate([[0], np.cumsum(cut)]).astype(np.int64)
            rows = np.concatenate([np.arange(w.offsets[b], w.offsets[b] + cut[b])
                                   for b in range(w.n_seq)])
            pdb = h.DeviceBatch(w.obs[rows], offs, dtype=np.float64 if prec == "f64" else np.float32)
            scale = T_max / plain_t
            plain_note = (f"timed on the batch cut to its first {plain_t} steps per sequence, "
                          f"scaled by {scale:.1f} (linear in the longest sequence)")
        else:
            pdb = db
        pws = h._ws(h.hmm_workspace_size("estep", dm, pdb, pprec))

        def pstep():
            h.hmm_estep_stats(dm, pdb, pprec, stats, loglik, status, pws)

        pstep()
        torch.cuda.synchronize()
        log("plain warm-up done")
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.plain_steps):
            pstep()
        t1.record()
        torch.cuda.synchronize()
        plain_ms = t0.elapsed_time(t1) / args.plain_steps * scale
        log(f"plain: {plain_ms:.3f} ms per E-step")
        del pws

    # Baum-Welch: E-step + FP64 M-step of the family (Gamma Newton, Student-t ECM),
    # em_iters iterations
    # captured once in a HIP graph and replayed
    em = None
    if args.em_iters > 0:
        m0 = workloads.perturb(w.model, np.random.default_rng(1))
        em_model = h.DeviceModel.from_model(m0)
        K = args.em_iters
        em_stats = torch.zeros((K, S), dtype=torch.float64, device="cuda")
        start = [t.clone() for t in (em_model.log_pi, em_model.log_A, em_model.theta)]

        def em_loop():
            for k in range(K):
                h.em_iteration(em_model, db, prec, em_stats[k], loglik, status, ws)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            em_loop()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            em_loop()
        for dst, src in zip((em_model.log_pi, em_model.log_A, em_model.theta), start):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        em_ms = e0.elapsed_time(e1)
        traj = em_stats[:, 0].cpu().numpy()
        log(f"EM graph: {em_ms / K:.3f} ms per iteration")
        em = {"iterations": K, "ms_total": em_ms, "ms_per_iteration": em_ms / K,
              "transitions_per_s": K * w.transitions / (em_ms / 1e3),
              "loglik_first": float(traj[0]), "loglik_last": float(traj[-1]),
              "loglik_non_decreasing": bool(np.all(np.diff(traj) >= -1e-6 * np.abs(traj[1:])))}

    value = w.transitions / (ms / 1e3)
    dom = max(kt, key=lambda k: kt[k]["ms_total"])
    fl = algorithmic_flops(dom, w)
    roof = None
    if fl is not None:
        ach = fl / (kt[dom]["ms_avg"] / 1e3) / 1e12
        # the scaled low-precision sweeps run their products on the matrix cores
        mfma = prec in ("bf16_scaled", "f16_scaled") and dom in ("block_fwd", "block_bwd")
        peak = (PEAK_BF16_MFMA_TFLOPS if mfma else
                PEAK_FP64_VALU_TFLOPS if prec == "f64" else PEAK_FP32_VALU_TFLOPS)
        roof = {"bound": "mfma" if mfma else "alu", "kernel": dom, "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": measured_traffic(dom, args.workload),
                "kernel_ms_avg": kt[dom]["ms_avg"]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "transitions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "eager_ms_per_step": eager_ms,
        "timing": ("eager calls (no graph)" if args.eager_only else
                   "E-steps replayed from one captured HIP graph; eager figure beside it"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "bf16_scaled": "bf16", "f16_scaled": "f16"}[prec],
        "data": "synthetic",
        "config": {"workload": wl_name, "global_batch": w.n_seq, "total_steps": w.total_steps,
                   "transitions_per_step": w.transitions, "precision": prec},
        "plain_gpu": None if plain_ms is None else {
            "value": w.transitions / (plain_ms / 1e3), "ms_per_step": plain_ms,
            "speedup": plain_ms / ms, "note": plain_note},
        "roofline": roof,
        "em_graph": em,
        "kernels": kt,
    }
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 256 MiB copied")
    if args.others > 0 and args.workload == "batched":
        out["other_workloads"] = other_workloads(h, workloads, args.others)
    if args.serving_seconds > 0:
        qps = [float(x) for x in args.serving_qps.split(",") if x]
        out["serving"] = serving_bench(h, workloads, qps, args.serving_seconds,
                                       streams=args.serving_streams)
        log("serving done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
