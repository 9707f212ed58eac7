"""Throughput of FastFCA-AS against conventional FCA EM on one MI355X.

A step is one whole separation job on the 10 s speech-scale workload
(I = J = 3 microphones/sources, F = 513 bins, N = 626 frames, 100 hybrid
iterations, complex64 data with FP32 arithmetic): reset the parameters to the
seeded initial point, run the 100 iterations (Section 4.3 of the paper),
evaluate the log-likelihood (eq. 14) and apply the multichannel Wiener filter
(eq. 3).  Inputs are resident in device memory before timing starts.

value = N * F * iterations / (seconds per step), in time-frequency-point
iterations per second.  The same job with the conventional FCA EM algorithm
(Section 3.3) is timed beside it on the same GPU.  The JSON line also
carries, each with its own roofline, the same job at the paper's shape
(I = J = 3, F = 512, N = 249, 20 iterations) and at the two 60 s
large-array shapes (I = 6, J = 4 and I = 8, J = 6; F = 1025, N = 3750,
50 iterations), the uneven batch (64 mixtures, 30 iterations per step), the
forward + reverse pass of the unrolled method, and the FP64 CPU oracle timed
on the host's cores (a process pool over the frequency bins, and one core).

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3]
       python bench.py --calibrate-copy     (plain copy of a known size, for
                                             scaling hardware byte counters)
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published
CPU_POOL_MAX = 16               # host cores that go with one GPU

METRIC = "TF-point-iters/s: FastFCA-AS vs plain FCA EM, 1 GPU, I=J=3, F=513"


def as_bytes_per_point_iter(I, J):
    """Algorithmic HBM bytes of one FastFCA-AS iteration per time-frequency
    point: read x (8I), read v (4J), write v (4J)."""
    return 8 * I + 8 * J


def as_flops_per_point_iter(I, J):
    """Algorithmic FP32 operations of one hybrid iteration per point:
    basis transform y = P^H x (8I^2), |y|^2 (3I), model variances, gains,
    posterior statistics and the v update (11IJ), lambda sums (2IJ + J),
    new variances and weights (2IJ + I), x x^H (3I + 3I(I-1)) and the I
    weighted covariance sums (2I^3)."""
    return 8 * I * I + 3 * I + 11 * I * J + 2 * I * J + J + 2 * I * J + I + 3 * I + 3 * I * (I - 1) + 2 * I ** 3


def fca_em_flops_per_point_iter(I, J):
    """Algorithmic FP32 operations of one conventional FCA EM iteration per
    point (complex multiply-add = 8 flops): model covariance (2JI^2), one
    Hermitian inverse (~4I^3 by Cholesky), per source the two products
    S_j C^-1 and (S_j C^-1) S_j (8I^3 + 4I^3), mu_j (8I^2), Rhat (6I^2),
    trace (4I^2) and the sum of eq. 10 (2I^2)."""
    return 2 * J * I * I + 4 * I ** 3 + J * (12 * I ** 3 + 20 * I * I)


# What each profiled kernel compiles from (the counters are void once these change).
RESIDENT_SOURCES = ("fca_resident.h", "fca_point.h", "fca_device.h", "fca_state.h")
STREAM_SOURCES = ("fca_kernels.h", "fca_pvariants.h", "fca_point.h", "fca_device.h", "fca_state.h")


def _sources_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1805_09498_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def _summary_fields(path):
    try:
        return dict(line.split(": ", 1) for line in open(path).read().splitlines()
                    if ": " in line and not line.startswith(" "))
    except OSError:
        return None


def profiled_traffic(workload, shape):
    """HBM bytes per launch of the frequency-resident kernel from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary (one value per launch
    shape), or None when the kernel sources changed since the counters were
    taken (source hash), or the workload or launch shape was not profiled."""
    fields = _summary_fields(os.path.join(ROOT, "profiles", f"k_as_resident_{workload}_traffic.txt"))
    if fields is None:
        return None
    key = (f"traffic_bytes_per_launch[waves={shape['waves_per_workgroup']} "
           f"bins_per_wg={shape['bins_per_workgroup']}]")
    if fields.get("source_sha256") != _sources_hash(RESIDENT_SOURCES) or fields.get("workload") != workload \
            or key not in fields:
        return None
    return float(fields[key])


def profiled_stream_traffic(workload):
    """HBM bytes per iteration of the streaming kernels (pass A + pass B +
    solve) from the committed counter summary, or None (see above)."""
    fields = _summary_fields(os.path.join(ROOT, "profiles", f"k_as_pass_{workload}_traffic.txt"))
    if fields is None or fields.get("source_sha256") != _sources_hash(STREAM_SOURCES) \
            or fields.get("workload") != workload or "traffic_bytes_per_iteration" not in fields:
        return None
    return float(fields["traffic_bytes_per_iteration"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="speech10s")
    ap.add_argument("--iters", type=int, default=None, help="override the workload's iteration count")
    ap.add_argument("--F", type=int, default=None, help="override the number of frequency bins")
    ap.add_argument("--N", type=int, default=None, help="override the number of frames")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--bins-per-wg", type=int, default=0)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--path", type=int, default=0)
    ap.add_argument("--split-streams", type=int, default=0,
                    help="streaming FastFCA-AS: streams the bins are split over (1..4; 0 = library default)")
    ap.add_argument("--sums-mfma", type=int, default=-1,
                    help="streaming FastFCA-AS above I = 4: pass B's eq. 23 sums on the vector units (0) or the "
                         "matrix cores (1 = 16x16x4, 2 = 4x4x1 tiles); -1 = the library's default for I")
    ap.add_argument("--em-steps", type=int, default=3)
    ap.add_argument("--no-em", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload (no paper-shape, 60 s, batch legs)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--stream-ceilings", action="store_true",
                    help="print the GB/s of a 1.5 GB torch fill and copy, and exit")
    ap.add_argument("--batch", action="store_true",
                    help="uneven batch workload alone (64 mixtures, F=513, 30 iterations per step)")
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--no-fwd-bwd", action="store_true", help="skip the forward + reverse pass leg")
    ap.add_argument("--fwd-bwd-iters", type=int, default=20)
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="checkpoint interval of the forward + backward leg (0 = the whole run on the tape)")
    return ap.parse_args()


def calibrate_copy():
    import torch
    n = 256 << 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n, "bytes_written": n, "launches": 5}))


def stream_ceilings():
    """What plain torch streams reach on this GPU (HIP events, best of 5): a
    1.5 GB write-only fill and a 1.5 GB copy -- the practical ceilings beside
    the 8 TB/s peak for the output-bound Wiener filter."""
    import torch
    big = 3 << 29
    x = torch.empty(big // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    rates = {}
    for name, op, moved in (("fill_GBps", lambda: x.fill_(1.0), big), ("copy_GBps", lambda: y.copy_(x), 2 * big)):
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(); op(); e1.record(); torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        rates[name] = moved / (best * 1e-3) / 1e9
    print(json.dumps({"stream_ceilings": rates}))


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, on the host's cores.
# ---------------------------------------------------------------------------
_POOL_PROB = None     # the problem the pool's workers inherit (fork)


def _oracle_bins(job):
    """Worker: `iters` iterations of one method on bins [f0, f1) of the
    inherited problem, BLAS on one thread; returns the seconds it took."""
    method, f0, f1, iters = job
    import oracle
    from threadpoolctl import threadpool_limits
    p = _POOL_PROB
    x = p.x[f0:f1]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        if method == "as":
            v, lam, P = p.v0[f0:f1], p.lam0[f0:f1], p.P0[f0:f1]
            for _ in range(iters):
                v, lam, P = oracle.fastfca_as_step(x, v, lam, P)
        else:
            v, R = p.v0[f0:f1], oracle.as_spatial_cov(p.P0[f0:f1], p.lam0[f0:f1])
            for _ in range(iters):
                v, R = oracle.fca_em_step(x, v, R)
        return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, iters_as_pool=100, iters_em_pool=20, iters_as_one=20, iters_em_one=3):
    """The oracle timed on the host: frequency bins sharded over a process
    pool (one worker per available core, at most CPU_POOL_MAX, BLAS on one
    thread each), and on one core.  Runs before anything touches the GPU
    (the workers are forked)."""
    import multiprocessing as mp
    global _POOL_PROB
    _POOL_PROB = prob
    F, N, I, J = prob.shape
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(avail, CPU_POOL_MAX))
    edges = np.linspace(0, F, workers + 1).astype(int)

    def pool_rate(pool, method, iters):
        jobs = [(method, int(a), int(b), iters) for a, b in zip(edges[:-1], edges[1:]) if b > a]
        t0 = time.perf_counter()
        pool.map(_oracle_bins, jobs, chunksize=1)
        return N * F * iters / (time.perf_counter() - t0)

    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_oracle_bins, [("as", 0, 1, 1)] * workers)          # start every worker
        as_pool = pool_rate(pool, "as", iters_as_pool)
        em_pool = pool_rate(pool, "em", iters_em_pool)
    as_one = N * F * iters_as_one / _oracle_bins(("as", 0, F, iters_as_one))
    em_one = N * F * iters_em_one / _oracle_bins(("em", 0, F, iters_em_one))
    return {
        "value": as_pool, "unit": "TF-point-iters/s", "cores": workers, "kind": "oracle",
        "sample": (f"FastFCA-AS oracle (numpy FP64), {iters_as_pool} iterations of all {F} bins of the "
                   f"{F}x{N} I={I} J={J} workload sharded over {workers} forked processes, BLAS on one "
                   f"thread each; also FCA EM oracle {iters_em_pool} iterations on the pool and both methods "
                   f"on one core ({iters_as_one} and {iters_em_one} iterations)"),
        "host_cpu": _cpu_model(), "host_cores_available": avail,
        "fca_em_value": em_pool, "one_core": {"value": as_one, "fca_em_value": em_one},
    }


# ---------------------------------------------------------------------------
# GPU legs.
# ---------------------------------------------------------------------------
def upload(prob):
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(prob.x.astype(np.complex64)).to(dev),
            torch.from_numpy(prob.v0.astype(np.float32)).to(dev),
            torch.from_numpy(prob.lam0.astype(np.float32)).to(dev),
            torch.from_numpy(prob.P0.astype(np.complex64)).to(dev))


def timed_job(ff, tens, method, iters, n_steps, n_warm, opts=None):
    """Whole jobs (reset, iterations, log-likelihood into device memory,
    Wiener filter) back to back; returns wall ms per job, event-timed ms of
    the iterate call, the last log-likelihood and the launch shape used."""
    import torch
    x, v0, lam0, P0 = tens
    F, N, I = x.shape
    J = v0.shape[2]
    out = torch.empty((J, F, N, I), dtype=torch.complex64, device=x.device)
    ctx = ff.fca_init(method, x, v0, lam0, P0)
    for k, val in (opts or {}).items():
        ff.fca_set_option(ctx, k, val)
    if method == ff.FCA_METHOD_AS:
        iterate = ff.fastfca_as_iterate
        reset = (v0, lam0, P0)
    else:
        iterate = ff.fca_em_iterate
        _, _, R_init = ff.fca_get_params(ctx)
        reset = (v0, None, R_init.clone())
    # events on the library's stream (the context was created on the current stream)
    stream = torch.cuda.current_stream()
    events = []
    ll = torch.empty((1,), dtype=torch.float64, device=x.device)

    def step(record):
        ff.fca_set_params(ctx, *reset)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        iterate(ctx, iters)
        e1.record(stream)
        # the job's log-likelihood stays in device memory like its separated
        # images, so jobs queue back to back without a host round trip
        ff.fca_loglik_device(ctx, ll)
        ff.fca_wiener_separate(ctx, out)
        if record:
            events.append((e0, e1))

    for _ in range(n_warm):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L = float(ll.item())
    it_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    shape = {"waves_per_workgroup": ff.fca_get_option(ctx, "last_waves"),
             "bins_per_workgroup": ff.fca_get_option(ctx, "last_bins_per_wg")}
    ff.fca_destroy(ctx)
    del out
    return (t1 - t0) * 1e3 / n_steps, it_ms, L, shape


def roofline_for(I, J, pts, it_ms, shape, workload):
    """Roofline object of a FastFCA-AS iteration launch set: the
    frequency-resident kernel is VALU-bound (FP32 vector peak); the
    streaming passes are measured against the HBM peak with the algorithmic
    8I + 8J bytes per point-iteration."""
    flops = as_flops_per_point_iter(I, J) * pts
    bytes_alg = as_bytes_per_point_iter(I, J) * pts
    tflops = flops / (it_ms * 1e-3) / 1e12
    gbs = bytes_alg / (it_ms * 1e-3) / 1e9
    resident = shape["waves_per_workgroup"] > 0
    if resident:
        r = {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": profiled_traffic(workload, shape),
             "kernel": "k_as_resident (frequency-resident; all iterations of a step in one launch)"}
    else:
        per_it = profiled_stream_traffic(workload)
        r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
             "traffic": None if per_it is None else per_it,
             "traffic_unit": "bytes per iteration (all streaming launches of one iteration)",
             "kernel": "k_as_pass_a + k_as_pass_b + k_as_solve per iteration",
             "achieved_TFLOPs": tflops}
    r.update({"kernel_ms": it_ms, "algorithmic_GBps": gbs, "algorithmic_hbm_frac": gbs / HBM_PEAK_GBS,
              "launch_shape": shape})
    return r


def workload_leg(ff, name, steps, warmup, em_steps):
    """The separation job of one named workload with both methods."""
    from paper_1805_09498_amd import synth
    cfg = synth.CONFIGS[name]
    I, J, F, N, iters = cfg["I"], cfg["J"], cfg["F"], cfg["N"], cfg["iters"]
    prob = synth.make_config(name).rounded_c64()
    tens = upload(prob)
    del prob
    ms, it_ms, L, shape = timed_job(ff, tens, ff.FCA_METHOD_AS, iters, steps, warmup)
    pts = N * F * iters
    leg = {"workload": f"{name}: I={I}, J={J}, F={F}, N={N}, {iters} iterations + log-likelihood + Wiener filter "
                       "per step, complex64",
           "value": pts / (ms * 1e-3), "unit": "TF-point-iters/s", "ms_per_step": ms, "steps": steps,
           "iterate_ms": it_ms, "loglik": L, "roofline": roofline_for(I, J, pts, it_ms, shape, name)}
    if em_steps > 0:
        ms_em, it_ms_em, L_em, shape_em = timed_job(ff, tens, ff.FCA_METHOD_EM, iters, em_steps, 1)
        leg["fca_em"] = {"value": pts / (ms_em * 1e-3), "ms_per_step": ms_em, "iterate_ms": it_ms_em,
                         "loglik": L_em, "launch_shape": shape_em,
                         "achieved_TFLOPs": fca_em_flops_per_point_iter(I, J) * pts / (it_ms_em * 1e-3) / 1e12}
        leg["speedup_vs_fca_em"] = leg["value"] / leg["fca_em"]["value"]
    return leg


def batch_leg(ff, steps, warmup, iters=30, graph=1, queues=(0, 1)):
    """Uneven batch: 64 mixtures (N ~ U[200, 2000], I in {2,3,4,6},
    J ~ U[2, I+1], F = 513), `iters` FastFCA-AS iterations per step through
    the batch API (one launch per (I, J) group, replayed as a HIP graph)."""
    import torch
    from paper_1805_09498_amd import synth
    probs = [p.rounded_c64() for p in synth.make_batch(n_mix=64, F=513, seed=4000)]
    shapes = [p.shape for p in probs]
    tens, init = [], []
    for p in probs:
        t = upload(p)
        tens.append(t)
        init.append((t[1].clone(), t[2].clone(), t[3].clone()))
    del probs
    stream = torch.cuda.current_stream()
    b = ff.fca_batch_init(tens)
    ff.fca_batch_set_option(b, "graph", graph)
    ctxs = [ff.fca_batch_context(b, m) for m in range(len(shapes))]

    def step():
        for c, (v0, l0, P0) in zip(ctxs, init):
            ff.fca_set_params(c, v0, l0, P0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ff.fca_batch_iterate(b, iters)
        e1.record(stream)
        return e0, e1

    def timed():
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ev.append(step())
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, float(np.mean([a.elapsed_time(c) for a, c in ev]))

    # one workgroup per (mixture, bin) tile (the default), then the
    # persistent work-queue form of the same launches
    per_queue = {}
    for q in queues:
        ff.fca_batch_set_option(b, "queue", q)
        per_queue[q] = timed()
    ms, it_ms = per_queue[queues[0]]
    pts = sum(s[0] * s[1] for s in shapes) * iters
    groups = []
    for g in range(ff.fca_batch_get_option(b, "groups")):
        groups.append({k: ff.fca_batch_get_option(b, "group_" + k, g) for k in ("I", "J", "tiles", "waves", "queued")})
    flops = sum(as_flops_per_point_iter(s[2], s[3]) * s[0] * s[1] for s in shapes) * iters
    bytes_alg = sum(as_bytes_per_point_iter(s[2], s[3]) * s[0] * s[1] for s in shapes) * iters
    tflops = flops / (it_ms * 1e-3) / 1e12
    ff.fca_batch_destroy(b)
    return {"workload": "64 mixtures, F=513, N~U[200,2000], I in {2,3,4,6}, J~U[2,I+1], "
                        f"{iters} iterations per step (parameters reset each step)",
            "value": pts / (ms * 1e-3), "unit": "TF-point-iters/s", "ms_per_step": ms, "iterate_ms": it_ms,
            "steps": steps, "graph": bool(graph), "launches_per_step": len(groups),
            "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                         "algorithmic_GBps": bytes_alg / (it_ms * 1e-3) / 1e9,
                         "kernel": "k_as_resident_batch, one launch per (I, J) group"},
            "work_queue": {"value": pts / (per_queue[1][0] * 1e-3), "ms_per_step": per_queue[1][0],
                           "iterate_ms": per_queue[1][1],
                           "kernel": "k_as_resident_batch_q: persistent workgroups, device tile counter"}
            if 1 in per_queue and queues[0] != 1 else None,
            "groups": groups}


def batch_main(args):
    from paper_1805_09498_amd import fastfca as ff
    leg = batch_leg(ff, args.steps, args.warmup, args.iters or 30, args.graph)
    leg.update({"metric": "TF-point-iters/s, uneven batch (FastFCA-AS)", "n_gpus": 1, "warmup": args.warmup,
                "higher_is_better": True, "dtype": "f32", "data": "synthetic"})
    print(json.dumps(leg))


def fwd_bwd_leg(ff, x, v0, lam0, P0, n_iter, every, steps, warmup):
    """Recorded forward (n_iter iterations, a checkpoint every `every`, Wiener
    filter) and the full reverse pass for a fixed seeded dL/d(images), from the
    same initial point each step.  Times per step and per half (HIP events on
    the current stream, the library's stream here)."""
    import torch
    F, N, I = x.shape
    J = v0.shape[2]
    g = torch.randn((J, F, N, I), dtype=torch.complex64, device=x.device,
                    generator=torch.Generator(device=x.device).manual_seed(0))
    ctx = ff.fca_init(ff.FCA_METHOD_AS, x, v0, lam0, P0)
    stream = torch.cuda.current_stream()
    ev = []

    def step(record):
        ff.fca_set_params(ctx, v0, lam0, P0)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        ff.fastfca_as_forward(ctx, n_iter, every)
        e1.record(stream)
        ff.fastfca_as_backward(ctx, g)
        e2.record(stream)
        if record:
            ev.append((e0, e1, e2))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    fwd = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    bwd = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    ff.fca_destroy(ctx)
    return {"workload": f"I={I}, J={J}, F={F}, N={N}: {n_iter} recorded FastFCA-AS iterations + Wiener "
                        f"filter, then the reverse pass (hand-written adjoints, checkpoint every {every}) "
                        "for a fixed dL/d(images) to x, v0, lambda0, P0",
            "value": N * F * n_iter / (ms * 1e-3), "unit": "TF-point-iters/s (forward + backward)",
            "ms_per_step": ms, "forward_ms": fwd, "backward_ms": bwd}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; the frequency bins shard across "
                                   "GPUs without communication, but no multi-GPU run is implemented"}))
        sys.exit(2)
    if args.batch:
        batch_main(args)
        return
    if args.stream_ceilings:
        stream_ceilings()
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    from paper_1805_09498_amd import synth

    cfg = dict(synth.CONFIGS[args.config])
    iters = args.iters or cfg["iters"]
    over = {k: getattr(args, k) for k in ("F", "N") if getattr(args, k)}
    cfg.update(over)
    I, J, F, N = cfg["I"], cfg["J"], cfg["F"], cfg["N"]
    prob = synth.make_config(args.config, **over).rounded_c64()
    # the CPU baseline forks its workers before anything initialises the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(prob)

    from paper_1805_09498_amd import fastfca as ff
    tens = upload(prob)
    opts = {"waves": args.waves, "bins_per_wg": args.bins_per_wg, "path": args.path, "autotune": args.autotune}
    if args.split_streams:
        opts["split_streams"] = args.split_streams
    if args.sums_mfma >= 0:
        opts["sums_mfma"] = args.sums_mfma
    ms_as, it_ms_as, L_as, shape_as = timed_job(ff, tens, ff.FCA_METHOD_AS, iters, args.steps, args.warmup, opts)
    pts = N * F * iters
    value = pts / (ms_as * 1e-3)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "TF-point-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_as,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}{' (overridden)' if over else ''}: I={I}, J={J}, F={F}, N={N}, {iters} FastFCA-AS iterations "
                               f"+ log-likelihood + Wiener filter per step, complex64",
                   "I": I, "J": J, "F": F, "N": N, "iterations": iters, "parallelism": "1 GPU"},
    }
    # dominant kernel: the iteration launch(es) timed by events on the library's stream
    res["roofline"] = roofline_for(I, J, pts, it_ms_as, shape_as, args.config if not over else "")
    if shape_as["waves_per_workgroup"] > 0 and iters > 1024:
        res["roofline"]["traffic"] = None
    res["loglik"] = L_as
    if not args.no_em:
        ms_em, it_ms_em, L_em, shape_em = timed_job(ff, tens, ff.FCA_METHOD_EM, iters, args.em_steps, 1)
        v_em = pts / (ms_em * 1e-3)
        res["fca_em"] = {"value": v_em, "ms_per_step": ms_em, "iterate_ms": it_ms_em, "loglik": L_em,
                         "launch_shape": shape_em,
                         "achieved_TFLOPs": fca_em_flops_per_point_iter(I, J) * pts / (it_ms_em * 1e-3) / 1e12}
        res["speedup_vs_fca_em"] = value / v_em
        # the paper's own figure, for context only (another machine, another
        # implementation, a different workload)
        res["paper_speedup_context"] = {
            "speedup_vs_fca": "over 420x (parameter estimation, ratio of real-time factors)",
            "hardware": "Intel i7-2600 3.4 GHz CPU, MATLAB R2013a",
            "workload": "I=J=3, F=512, 8 s speech mixtures, 20 iterations, averaged over trials",
            "source": "Section 5 (Figure of the real-time factor) and the abstract"}
    if not args.no_fwd_bwd:
        # By default one segment: the forward run records every state (a tape
        # of about 0.1 GB at this shape, which HBM holds easily), so the
        # reverse pass recomputes none; the same job with a checkpoint every
        # 5 iterations (three segments rebuilt) is reported beside it.
        every = args.ckpt_every or args.fwd_bwd_iters
        res["fwd_bwd"] = fwd_bwd_leg(ff, *tens, args.fwd_bwd_iters, every, max(3, args.steps // 4), 2)
        res["fwd_bwd"]["checkpoint_every_5"] = fwd_bwd_leg(ff, *tens, args.fwd_bwd_iters, 5,
                                                           max(3, args.steps // 4), 2)
    if not args.no_extra:
        res["paper_shape"] = workload_leg(ff, "paper", max(3, args.steps // 2), 2, 2 if not args.no_em else 0)
        for name in ("long6x4", "long8x6"):
            res[name] = workload_leg(ff, name, 2, 1, 1 if not args.no_em else 0)
        res["batch"] = batch_leg(ff, 3, 1)
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res))


if __name__ == "__main__":
    main()
