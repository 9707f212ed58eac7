"""Throughput of FastFCA-AS against conventional FCA EM on one MI355X.

A step is one whole separation job on the 10 s speech-scale workload
(I = J = 3 microphones/sources, F = 513 bins, N = 626 frames, 100 hybrid
iterations, complex64 data with FP32 arithmetic): reset the parameters to the
seeded initial point, run the 100 iterations (Section 4.3 of the paper),
evaluate the log-likelihood (eq. 14) and apply the multichannel Wiener filter
(eq. 3).  Inputs are resident in device memory before timing starts.

value = N * F * iterations / (seconds per step), in time-frequency-point
iterations per second.  The same job with the conventional FCA EM algorithm
(Section 3.3) is timed beside it on the same GPU, and the FP64 CPU oracle is
timed on a bounded sample on the host.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3]
       python bench.py --calibrate-copy     (plain copy of a known size, for
                                             scaling hardware byte counters)
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published

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


KERNEL_SOURCES = ("fca_resident.h", "fca_point.h", "fca_device.h", "fca_state.h")  # what k_as_resident compiles from
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_as_resident_speech10s_traffic.txt")


def profiled_traffic(workload, shape):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (one value per launch shape), or
    None when the kernel sources changed since the counters were taken
    (source hash), or the workload or launch shape was not profiled."""
    import hashlib
    try:
        fields = dict(line.split(": ", 1) for line in open(TRAFFIC_FILE).read().splitlines()
                      if ": " in line and not line.startswith(" "))
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1805_09498_amd", "csrc", f), "rb").read())
    key = (f"traffic_bytes_per_launch[waves={shape['waves_per_workgroup']} "
           f"bins_per_wg={shape['bins_per_workgroup']}]")
    if fields.get("source_sha256") != h.hexdigest() or fields.get("workload") != workload or key not in fields:
        return None
    return float(fields[key])


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
    ap.add_argument("--em-steps", type=int, default=3)
    ap.add_argument("--no-em", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="uneven batch workload instead (64 mixtures, F=513, 30 iterations per step)")
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--no-fwd-bwd", action="store_true", help="skip the forward + reverse pass leg")
    ap.add_argument("--fwd-bwd-iters", type=int, default=20)
    ap.add_argument("--ckpt-every", type=int, default=5)
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


def cpu_baseline(prob, iters_as=60, iters_em=8):
    """The FP64 oracle as it stands, single-threaded, on the same rounded
    inputs: a bounded number of iterations of each method."""
    import oracle
    from threadpoolctl import threadpool_limits
    F, N, I, J = prob.shape
    out = {}
    with threadpool_limits(1):
        v, lam, P = prob.v0, prob.lam0, prob.P0
        t0 = time.perf_counter()
        for _ in range(iters_as):
            v, lam, P = oracle.fastfca_as_step(prob.x, v, lam, P)
        t_as = time.perf_counter() - t0
        R = oracle.as_spatial_cov(prob.P0, prob.lam0)
        v = prob.v0
        t0 = time.perf_counter()
        for _ in range(iters_em):
            v, R = oracle.fca_em_step(prob.x, v, R)
        t_em = time.perf_counter() - t0
    out["value"] = N * F * iters_as / t_as
    out["unit"] = "TF-point-iters/s"
    out["cores"] = 1
    out["kind"] = "oracle"
    out["sample"] = (f"FastFCA-AS oracle, {iters_as} of the workload's iterations on all {F} bins "
                     f"({t_as:.1f} s); FCA EM oracle {iters_em} iterations ({t_em:.1f} s) -> "
                     f"{N * F * iters_em / t_em:.4g} TF-point-iters/s; numpy FP64, 1 thread")
    out["fca_em_value"] = N * F * iters_em / t_em
    return out


def batch_main(args):
    """Uneven batch: 64 mixtures (N ~ U[200, 2000], I in {2,3,4,6},
    J ~ U[2, I+1], F = 513), 30 FastFCA-AS iterations per step through the
    batch API (one launch per (I, J) group, replayed as a HIP graph)."""
    import torch
    from paper_1805_09498_amd import fastfca as ff
    from paper_1805_09498_amd import synth
    probs = [p.rounded_c64() for p in synth.make_batch(n_mix=64, F=513, seed=4000)]
    dev = torch.device("cuda:0")
    tens, init = [], []
    for p in probs:
        t = (torch.from_numpy(p.x.astype(np.complex64)).to(dev), torch.from_numpy(p.v0.astype(np.float32)).to(dev),
             torch.from_numpy(p.lam0.astype(np.float32)).to(dev), torch.from_numpy(p.P0.astype(np.complex64)).to(dev))
        tens.append(t)
        init.append((t[1].clone(), t[2].clone(), t[3].clone()))
    stream = torch.cuda.current_stream()
    b = ff.fca_batch_init(tens)
    ff.fca_batch_set_option(b, "graph", args.graph)
    ctxs = [ff.fca_batch_context(b, m) for m in range(len(probs))]
    iters = args.iters or 30

    def step():
        for c, (v0, l0, P0) in zip(ctxs, init):
            ff.fca_set_params(c, v0, l0, P0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ff.fca_batch_iterate(b, iters)
        e1.record(stream)
        return e0, e1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    it_ms = float(np.mean([a.elapsed_time(c) for a, c in ev]))
    pts = sum(p.shape[0] * p.shape[1] for p in probs) * iters
    groups = []
    for g in range(ff.fca_batch_get_option(b, "groups")):
        groups.append({k: ff.fca_batch_get_option(b, "group_" + k, g) for k in ("I", "J", "tiles", "waves")})
    flops = sum(as_flops_per_point_iter(p.shape[2], p.shape[3]) * p.shape[0] * p.shape[1] for p in probs) * iters
    print(json.dumps({
        "metric": "TF-point-iters/s, uneven batch (FastFCA-AS)", "value": pts / (ms * 1e-3),
        "unit": "TF-point-iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "iterate_ms": it_ms, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 mixtures, F=513, N~U[200,2000], I in {2,3,4,6}, J~U[2,I+1], "
                               f"{iters} iterations per step (parameters reset each step)",
                   "graph": bool(args.graph)},
        "achieved_TFLOPs": flops / (it_ms * 1e-3) / 1e12, "groups": groups}))


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
    if args.batch and args.gpus == 1:
        batch_main(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; the frequency bins shard across "
                                   "GPUs without communication, but no multi-GPU run is implemented"}))
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        calibrate_copy()
        return
    from paper_1805_09498_amd import fastfca as ff
    from paper_1805_09498_amd import synth

    cfg = dict(synth.CONFIGS[args.config])
    iters = args.iters or cfg["iters"]
    over = {k: getattr(args, k) for k in ("F", "N") if getattr(args, k)}
    cfg.update(over)
    I, J, F, N = cfg["I"], cfg["J"], cfg["F"], cfg["N"]
    prob = synth.make_config(args.config, **over).rounded_c64()
    dev = torch.device("cuda:0")
    x = torch.from_numpy(prob.x.astype(np.complex64)).to(dev)
    v0 = torch.from_numpy(prob.v0.astype(np.float32)).to(dev)
    lam0 = torch.from_numpy(prob.lam0.astype(np.float32)).to(dev)
    P0 = torch.from_numpy(prob.P0.astype(np.complex64)).to(dev)
    out = torch.empty((J, F, N, I), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()

    def timed_job(method, n_steps, n_warm):
        ctx = ff.fca_init(method, x, v0, lam0, P0)
        if method == ff.FCA_METHOD_AS:
            ff.fca_set_option(ctx, "waves", args.waves)
            ff.fca_set_option(ctx, "bins_per_wg", args.bins_per_wg)
            ff.fca_set_option(ctx, "path", args.path)
            ff.fca_set_option(ctx, "autotune", args.autotune)
            if args.split_streams:
                ff.fca_set_option(ctx, "split_streams", args.split_streams)
            iterate = ff.fastfca_as_iterate
            reset = (v0, lam0, P0)
        else:
            iterate = ff.fca_em_iterate
            _, _, R_init = ff.fca_get_params(ctx)
            reset = (v0, None, R_init.clone())
        events = []
        ll = torch.empty((1,), dtype=torch.float64, device=dev)

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
        return (t1 - t0) * 1e3 / n_steps, it_ms, L, shape

    ms_as, it_ms_as, L_as, shape_as = timed_job(ff.FCA_METHOD_AS, args.steps, args.warmup)
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
    flops = as_flops_per_point_iter(I, J) * pts
    bytes_alg = as_bytes_per_point_iter(I, J) * pts
    res["roofline"] = {
        "bound": "alu",
        "achieved": flops / (it_ms_as * 1e-3) / 1e12,
        "peak": FP32_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": flops / (it_ms_as * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
        "traffic": None,
        "kernel": ("k_as_resident (frequency-resident; all iterations of a step in one launch)"
                   if args.path != 2 else "k_as_pass_a + k_as_pass_b + k_as_solve per iteration"),
        "kernel_ms": it_ms_as,
        "algorithmic_GBps": bytes_alg / (it_ms_as * 1e-3) / 1e9,
        "algorithmic_hbm_frac": bytes_alg / (it_ms_as * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    res["roofline"]["launch_shape"] = shape_as
    if args.path != 2 and iters <= 1024:
        res["roofline"]["traffic"] = profiled_traffic(args.config, shape_as)
    res["loglik"] = L_as
    if not args.no_em:
        ms_em, it_ms_em, L_em, shape_em = timed_job(ff.FCA_METHOD_EM, args.em_steps, 1)
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
        res["fwd_bwd"] = fwd_bwd_leg(ff, x, v0, lam0, P0, args.fwd_bwd_iters, args.ckpt_every,
                                     max(3, args.steps // 4), 2)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
