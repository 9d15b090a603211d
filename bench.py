#!/usr/bin/env python3
"""Throughput of dual-domain CSC on one MI355X.

Workload (synthetic stand-in for the paper's grayscale image sets): N = 10
contrast-normalised 1/f images of 100 x 100 zero-padded to 128 x 128, K = 100
filters of 11 x 11, beta = 1, adaptive rho from 10.  One step is one outer
alternation of Alg. 1: 10 ADMM coding iterations (warm-started), the learning
subproblem (10 multiplier updates x 10 CG iterations, warm-started gamma) and
the objective.  Inputs are resident in HBM before timing starts.

Printed: one JSON line.  ``value`` = code-pixel-iterations per second over the
whole step (N * K * H * W * coding iterations / step time).  ``roofline``
covers learning pass A (with pass B, the largest shares of the step), its
launch duration measured with HIP events on its own stream during the timed
steps; ``roofline_extra`` gives the same for learning pass B and the fused
coding kernel.  ``traffic`` is taken from the committed rocprofv3 counter
summary when the library sources still match the ones it was measured on,
else null.  ``cpu_baseline`` times the FP64 oracle on a bounded sample of
the same step.

``--calibrate-copy MIB`` only runs a plain device copy of that size (the
reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters);
``--profile-leg`` runs only the timed calls of one leg (the step's coding
call, the batched leg, the plain solver of the differentiable leg or that
leg's forward + backward, the tensor or the variant legs), for kernel
traces and counter collection.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
TRACE_EVERY = 32  # timed steps time every 32nd launch of a traced kernel (from the first)
FP32_VECTOR_TFLOPS = 157.3     # MI355X fp32 vector (packed); 78.6 unpacked
FP64_VECTOR_TFLOPS = 78.6      # MI355X fp64 vector (and fp64 matrix)


def alg_bytes_per_iter(n, j, k, d):
    """Bytes one coding iteration must move: z read + write (float32), the
    filter spectra once (half spectra, complex64), per-image spectra."""
    return 8 * n * k * d + 4 * j * k * d + 12 * n * j * d


def alg_bytes_pass_a(n, j, k, h, w, m1, m2):
    """Bytes one learning pass A must move: the N x ceil(K/2) code pair spectra
    (4 N K D), the CG vector at the canonical half of the frequencies
    (8 N J (H/2+1) W) and its output, one M1 x M2 column-stage partial per
    row group of 256 / W canonical rows (8 J ceil(K/2) G M1 M2)."""
    p = (k + 1) // 2
    r = 256 // w
    g = (h // 2 + r) // r
    return 8 * n * p * h * w + 8 * n * j * (h // 2 + 1) * w + 8 * j * p * g * m1 * m2


def alg_bytes_pass_b(n, j, k, h, w):
    """Bytes one learning pass B must move: the code pair spectra (4 N K D),
    the projected filter spectra at the canonical frequencies (16 J P
    (H/2+1) W), the CG vector read and the result written (16 N J D)."""
    p = (k + 1) // 2
    return 8 * n * p * h * w + 16 * j * p * (h // 2 + 1) * w + 16 * n * j * h * w


def span_apply_flops(j, k, m1, m2):
    """Float64 flops of one product with the correlation table in the span
    form of the learning CG: every output tap of every filter sums over all
    filters and taps, (M w)_k(q) = sum_l sum_q' C_kl(q - q') w_l(q'), i.e.
    J K^2 (M1 M2)^2 multiply-adds."""
    return 2.0 * j * k * k * (m1 * m2) ** 2


def span_rows_flops(n, j, k, h, w, m2):
    """Float64 flops of the row stage of the correlation table for the pairs
    the learning call uses (code-code k <= l, code-x and code-gamma per
    channel, three per channel among x and gamma): per pair and frequency of
    the H/2+1 canonical rows, N complex multiply-adds for the sum over
    images and 2 M2 real multiply-adds per output lag pair (+-delta2)."""
    pairs = k * (k + 1) // 2 + 2 * j * k + 3 * j
    return 8.0 * pairs * (h // 2 + 1) * w * (n + m2)


def csrc_digest():
    """sha256 over the library sources and the build script with its
    compiler flags (what the kernels the counters describe are made of)."""
    import hashlib
    src = os.path.join(ROOT, "paper_1709_09479_amd", "csrc")
    h = hashlib.sha256()
    paths = [os.path.join(src, n) for n in sorted(os.listdir(src)) if n.endswith((".hip", ".hpp", ".inc", ".py"))]
    paths.append(os.path.join(ROOT, "paper_1709_09479_amd", "build.py"))
    for path in paths:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(kernel):
    """HBM bytes per launch (or per call, for a whole leg) of `kernel` from the
    counter summaries profiles/*_hbm_bytes.md (FETCH_SIZE and WRITE_SIZE in
    KiB, scaled by the factors a plain copy kernel gives), or None when the
    library sources have changed since the counters were taken."""
    import glob
    digest = csrc_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_bytes.md"))):
        kv, rows = {}, {}
        for ln in open(path).read().splitlines():
            ln = ln.strip()
            if ln.startswith(("csrc_sha256 = ", "fetch_scale = ", "write_scale = ")):
                key, val = ln.split(" = ", 1)
                kv[key] = val.strip()
            elif ln.startswith("kernel "):
                parts = ln.split()
                vals = dict(x.split("=") for x in parts[2:])
                rows[parts[1]] = (float(vals["fetch_kib"]), float(vals["write_kib"]))
        if kernel in rows and kv.get("csrc_sha256") == digest:
            fk, wk = rows[kernel]
            return 1024.0 * (fk * float(kv["fetch_scale"]) + wk * float(kv["write_scale"]))
    return None


def calibrate_copy(mib):
    """A plain device copy of `mib` MiB, three times (counter calibration)."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_mib": mib, "bytes_each_way": n * 4}))


def bench_coding(dc, synth, np, torch, calls=20):
    """The step's coding call alone (10 images 128^2, K = 100, beta = 1,
    adaptive rho from 10, 10 iterations from zero codes): one warm-up call
    and `calls` timed ones, for kernel traces and counter collection."""
    cfg = synth.CONFIGS["learn"]
    b, d0 = synth.make_inputs(cfg)
    bt = torch.from_numpy(b).cuda()
    d = torch.from_numpy(d0).cuda()
    run = lambda: dc.code(bt, d, cfg.beta, cfg.rho0, cfg.t_in, adaptive=True)
    return {"workload": "coding of the learning step's images: N=10 128x128, K=100 11x11, beta=1, adaptive rho "
                        "from 10, 10 iterations", "ms_per_call": timed_ms(torch, run, calls)}


def bench_batched(dc, synth, np, torch, n_images, plain=True, tune=True):
    """Ragged batch: 256 images with sides drawn from 48..256 (padded to the
    next power of two), K = 64 shared 11x11 filters, beta = 1, rho = 10,
    30 ADMM iterations; one csc_code_batched call replayed from its hipGraph,
    against the plain solver called once per image.  With `tune` the pairs
    per workgroup of each single-tile class are measured first
    (autotune_batched); without, the library's heuristic grouping is used
    (the counter runs, which must see the batched call's dispatches only)."""
    cfg = synth.CONFIGS["batched"]
    imgs, grids, d0 = synth.ragged_inputs(cfg, n=n_images)
    dev = torch.device("cuda:0")
    padded = []
    for im, g in zip(imgs, grids):
        t = torch.zeros((1,) + g, dtype=torch.float32)
        t[:, :im.shape[1], :im.shape[2]] = torch.from_numpy(im)
        padded.append(t.to(dev))
    dt = torch.from_numpy(d0).to(dev)
    pb = dc.PackedBatch(padded, cfg.k)
    classes = pb.classes(cfg.fsupp)
    z = torch.empty(pb.z_numel, dtype=torch.float32, device=dev)
    it = cfg.t_in
    # pairs per workgroup of each single-tile class, measured on this GPU
    t0 = time.perf_counter()
    ppg = dc.autotune_batched(pb, dt, cfg.beta, cfg.rho, iters=3, persist=False) if tune else None
    tune_s = time.perf_counter() - t0
    dc.code_batched(pb, dt, cfg.beta, cfg.rho, it, z=z, graph=True, ppg=ppg)   # capture + first replay
    torch.cuda.synchronize()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dc.code_batched(pb, dt, cfg.beta, cfg.rho, it, z=z, graph=True, ppg=ppg)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pix_pad = sum(g[0] * g[1] for g in grids)
    pix_raw = sum(im.shape[1] * im.shape[2] for im in imgs)
    bytes_iter = sum(alg_bytes_per_iter(c, 1, cfg.k, g[0] * g[1]) for g, c in classes)
    out = {
        "workload": "%d ragged images (sides 48..256, padded to powers of two), K=%d 11x11, beta=1, rho=10, "
                    "%d iterations, hipGraph replay; five launches per iteration over work lists spanning all "
                    "grid classes" % (len(imgs), cfg.k, it),
        "grid_classes": [[g[0], g[1], c] for g, c in classes],
        "pairs_per_workgroup": ppg,
        "autotune_s": tune_s,
        "launches_per_iteration": 5,
        "ms_per_call": ms,
        "cp_it_per_s_padded": cfg.k * pix_pad * it / (ms / 1e3),
        "cp_it_per_s_unpadded": cfg.k * pix_raw * it / (ms / 1e3),
        "alg_gbps": bytes_iter * it / (ms / 1e3) / 1e9,
    }
    traffic = counter_traffic("batched_call")
    out["measured_gbps"] = None if traffic is None else traffic / (ms / 1e3) / 1e9
    if not plain:
        return out
    # plain solver, one call per image
    stack = [p[None] for p in padded]
    dc.code(stack[0], dt, cfg.beta, cfg.rho, it)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record()
    for x in stack:
        dc.code(x, dt, cfg.beta, cfg.rho, it)
    p1.record()
    torch.cuda.synchronize()
    ms_plain = p0.elapsed_time(p1)
    out["plain_per_image_ms"] = ms_plain
    out["speedup_vs_plain"] = ms_plain / ms
    return out


def bench_backward(dc, synth, np, torch, reps=2, only_plain=False, only_fwd_bwd=False):
    """Differentiable form: N = 16 images 256x256, K = 100 filters 11x11,
    30 unrolled ADMM iterations with checkpoints every 5, loss of eq:CSC;
    forward + backward (gradients w.r.t. filters and beta) against the plain
    solver (csc_code, 30 iterations) on the same inputs."""
    cfg = synth.CONFIGS["unrolled"]
    b, d0 = synth.make_inputs(cfg)
    dev = torch.device("cuda:0")
    bt = torch.from_numpy(b).to(dev)
    d = torch.from_numpy(d0).to(dev)
    beta = torch.tensor(cfg.beta, dtype=torch.float64, requires_grad=True)

    def fwd_bwd():
        dd = d.clone().requires_grad_(True)
        z = dc.unrolled_code(bt, dd, beta, cfg.rho, cfg.t_in, 5)
        L = dc.csc_loss(bt, dd, z, beta)
        L.backward()
        return L

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    if only_fwd_bwd:
        return {"forward_backward_ms": timed(fwd_bwd, reps)}
    ms_plain = timed(lambda: dc.code(bt, d, cfg.beta, cfg.rho, cfg.t_in), reps)
    traffic = counter_traffic("unrolled_plain_call")
    alg = alg_bytes_per_iter(cfg.n, cfg.j, cfg.k, cfg.grid[0] * cfg.grid[1]) * cfg.t_in
    if only_plain:
        return {"plain_code_ms": ms_plain}
    ms_fwd = timed(lambda: dc.unrolled_code(bt, d, cfg.beta, cfg.rho, cfg.t_in, 5), reps)
    ms_fb = timed(fwd_bwd, reps)
    cpit = cfg.n * cfg.k * cfg.grid[0] * cfg.grid[1] * cfg.t_in
    return {
        "workload": "N=16 images 256x256, K=100 11x11, beta=1, rho=10, 30 unrolled iterations, checkpoint every 5",
        "plain_code_ms": ms_plain,
        "unrolled_forward_ms": ms_fwd,
        "forward_backward_ms": ms_fb,
        "backward_ms": ms_fb - ms_fwd,
        "plain_cp_it_per_s": cpit / (ms_plain / 1e3),
        "plain_alg_gbps": alg / (ms_plain / 1e3) / 1e9,
        "plain_measured_gbps": None if traffic is None else traffic / (ms_plain / 1e3) / 1e9,
        "forward_backward_vs_plain": ms_fb / ms_plain,
    }


def timed_ms(torch, fn, reps):
    """Average milliseconds of `fn` over `reps` calls after one untimed call
    (HIP events on the current stream)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_tensor(dc, synth, np, torch, reps=3):
    """Tensor CSC (Sec. 3.3): 32 RGB images 128x128 with K = 64 colour filters
    11x11x3 (beta 0.5, rho 10, 20 iterations), and the 16-frame RGB video
    volume 16x128x128 with K = 64 filters 3x11x11x3: one csc_code call each."""
    out = {}
    for name in ("tensor", "video"):
        cfg = synth.CONFIGS[name]
        b, d0 = synth.make_inputs(cfg)
        bt = torch.from_numpy(b).cuda()
        dt = torch.from_numpy(d0).cuda()
        ms = timed_ms(torch, lambda: dc.code(bt, dt, cfg.beta, cfg.rho, cfg.t_in), reps)
        D = int(np.prod(cfg.grid))
        out[name] = {
            "workload": "N=%d J=%d grid %s, K=%d filters %s, beta=%g, rho=%g, %d iterations" % (
                cfg.n, cfg.j, "x".join(map(str, cfg.grid)), cfg.k, "x".join(map(str, cfg.fsupp)), cfg.beta, cfg.rho,
                cfg.t_in),
            "ms_per_call": ms,
            "cp_it_per_s": cfg.n * cfg.k * D * cfg.t_in / (ms / 1e3),
            "alg_gbps": alg_bytes_per_iter(cfg.n, cfg.j, cfg.k, D) * cfg.t_in / (ms / 1e3) / 1e9,
        }
    return out


def bench_variants(dc, synth, np, torch, reps=3):
    """The two variants on the benchmark's images (10 x 128^2, 10 iterations,
    rho 10), each against the plain circular l1 solver on the same images:
    the nuclear-norm regulariser (K = 100 filters 11x11, beta = 1: code maps of
    rank 4..15 of 128) and the DCT-domain variant with symmetric boundaries
    (K = 100 whole-sample symmetric 11x11 filters from 6x6 quadrants,
    beta = 1).  The coding map kernel of each iteration is timed by the
    library's tracer at its own start and end (DCT) or around the map
    sequence (nuclear: back-projection, inverse FFT, thresholding, FFT)."""
    cfg = synth.CONFIGS["learn"]
    b, d0 = synth.make_inputs(cfg)
    bt = torch.from_numpy(b).cuda()
    dt = torch.from_numpy(d0).cuda()
    q = torch.from_numpy(synth.symmetric_quadrants(cfg.k, 1, (6, 6), 2100)).cuda()
    N, K, it = cfg.n, cfg.k, cfg.t_in
    D = cfg.grid[0] * cfg.grid[1]
    cpit = N * K * D * it
    alg = alg_bytes_per_iter(N, 1, K, D)
    ms_plain = timed_ms(torch, lambda: dc.code(bt, dt, 1.0, 10.0, it), reps)
    out = {"plain_l1_ms": ms_plain}
    for name, fn in (("nuclear", lambda: dc.code(bt, dt, 1.0, 10.0, it, reg="nuclear")),
                     ("dct", lambda: dc.code_dct(bt, q, 1.0, 10.0, it))):
        fn()
        torch.cuda.synchronize()
        dc.trace_enable(True, every=1)
        ms = timed_ms(torch, fn, reps)
        dc.trace_enable(False)
        maps_ms, maps_cnt = dc.trace_read(dc.TRACE_CODE_MAPS)
        avg = maps_ms / max(1, maps_cnt)
        out[name] = {
            "ms_per_call": ms,
            "cp_it_per_s": cpit / (ms / 1e3),
            "vs_plain_l1": ms / ms_plain,
            "map_work_avg_ms": avg,
            "map_work_alg_gbps": alg / (avg / 1e3) / 1e9,
        }
    out["workload"] = ("10 images 128x128, 10 iterations, rho 10: nuclear norm (K=100 11x11, beta 1) and DCT "
                       "symmetric boundaries (K=100 symmetric 11x11, beta 1) against the circular l1 solver")
    return out


def cpu_all_cores(n_images, procs):
    """The oracle's coding of the benchmark's first `n_images` images (10
    ADMM iterations, adaptive rho, one image per task, as the coding problem
    separates over images) in `procs` worker processes.  Runs in a child
    process that never touches the GPU; prints one JSON object."""
    import multiprocessing as mp

    import numpy as np

    import synth
    cfg = synth.CONFIGS["learn"]
    b, d0 = synth.make_inputs(cfg)
    tasks = [(b[i:i + 1], d0, cfg.beta, cfg.rho0, cfg.t_in) for i in range(n_images)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        pool.map(_cpu_code_one, tasks)
    t = time.perf_counter() - t0
    D = cfg.grid[0] * cfg.grid[1]
    print(json.dumps({"value": n_images * cfg.k * D * cfg.t_in / t, "seconds": t, "procs": procs}))


def _cpu_code_one(task):
    import oracle
    b, d0, beta, rho, iters = task
    oracle.code(b, d0, beta, rho, iters, adaptive=True)
    return 0


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_sweep_point(dc, synth, np, torch, cfg, steps=5, conv_steps=30):
    """One point of a scaling sweep: the time of one outer step of the
    alternation at fixed counts (coding, learning, objective; median, p10,
    p90 over `steps` steps after one warm-up step), and the time to
    convergence of the convergence-driven alternation (tau = 1e-3 on the
    relative change of the objective, ADMM stopped at an RMS residual of 1e-3
    of the images' RMS within 100 iterations, CG at a relative residual of
    1e-3 within 50 steps, at most `conv_steps` outer steps)."""
    b, d0 = synth.make_inputs(cfg)
    dev = torch.device("cuda:0")
    bt = torch.from_numpy(b).to(dev)
    N, J, K = b.shape[0], cfg.j, cfg.k
    D = int(np.prod(cfg.grid))
    adaptive = cfg.rho is None
    rho0 = cfg.rho0 if adaptive else cfg.rho
    st = {"d": torch.from_numpy(d0).to(dev), "z": None, "theta": None, "gamma": None,
          "mu": torch.ones(K, dtype=torch.float32, device=dev),
          "rho": torch.full((N,), rho0, dtype=torch.float32, device=dev)}

    def step():
        st["z"], st["theta"], _, st["rho"] = dc.code(bt, st["d"], cfg.beta, st["rho"], cfg.t_in, z=st["z"],
                                                     theta=st["theta"], adaptive=adaptive, want_theta=True)
        st["d"], st["mu"], st["gamma"] = dc.learn(bt, st["z"], cfg.fsupp, st["mu"], st["gamma"], cfg.learn_inner,
                                                  cfg.learn_cg, out=st["d"])
        st["obj"] = dc.objective(bt, st["d"], st["z"], cfg.beta)

    step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    density = float(torch.count_nonzero(st["z"]).item()) / st["z"].numel()
    del st

    tol = 1e-3 * float(np.sqrt(np.mean(b.astype(np.float64) ** 2)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = dc.learn_dictionary(bt, torch.from_numpy(d0).to(dev), cfg.beta, rho0, 100, conv_steps,
                              cfg.learn_inner, 50, adaptive=adaptive, tau=1e-3, tol=tol, cg_tol=1e-3)
    torch.cuda.synchronize()
    conv_s = time.perf_counter() - t0
    code_its = [int(n) for n in out["coding_iters"]]
    cg = [int(c) for counts in out["cg_counts"] for c in counts]
    return {
        "point": cfg.name, "n": N, "j": J, "k": K, "grid": list(cfg.grid), "fsupp": list(cfg.fsupp),
        "beta": cfg.beta, "rho": "adaptive from %g" % rho0 if adaptive else rho0, "t_in": cfg.t_in,
        "learn": [cfg.learn_inner, cfg.learn_cg],
        "outer_step_ms": {"median": float(np.median(ms)), "p10": float(np.percentile(ms, 10)),
                          "p90": float(np.percentile(ms, 90))},
        "cp_it_per_s": N * K * D * cfg.t_in / (float(np.median(ms)) / 1e3),
        "code_density": density,
        "convergence": {"seconds": conv_s, "outer_steps": int(out["steps"]), "admm_iters": code_its,
                        "cg_steps_total": int(sum(cg)), "objective": float(out["objectives"][-1].item())},
    }


def run_sweeps(names):
    import numpy as np
    import torch

    import paper_1709_09479_amd as dc
    import synth

    dc.load()
    for name in names:
        for cfg in synth.SWEEPS[name]:
            r = bench_sweep_point(dc, synth, np, torch, cfg)
            r["sweep"] = name
            print(json.dumps(r), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-images", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--batched-images", type=int, default=256)
    ap.add_argument("--no-tensor", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-all-cores", type=int, default=0, metavar="PROCS", help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB")
    ap.add_argument("--profile-leg", choices=["coding", "batched", "unrolled-plain", "unrolled", "tensor", "variants"],
                    default=None,
                    help="run only the timed calls of one leg (for counter collection)")
    ap.add_argument("--sweep", default=None, metavar="NAMES",
                    help="comma-separated scaling sweeps (gray_K, gray_N, rgb_K, rgb_N, video_K, or all): "
                         "one JSON line per point instead of the benchmark line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the build targets a single MI355X); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.cpu_all_cores > 0:
        cpu_all_cores(10, args.cpu_all_cores)
        return
    if args.calibrate_copy > 0:
        calibrate_copy(args.calibrate_copy)
        return
    if args.sweep:
        import synth
        names = list(synth.SWEEPS) if args.sweep == "all" else args.sweep.split(",")
        unknown = [n for n in names if n not in synth.SWEEPS]
        if unknown:
            print("unknown sweep(s): %s" % ", ".join(unknown), file=sys.stderr)
            sys.exit(2)
        run_sweeps(names)
        return

    import numpy as np
    import torch

    import paper_1709_09479_amd as dc
    import synth

    dc.load()
    if args.profile_leg == "coding":
        print(json.dumps(bench_coding(dc, synth, np, torch)))
        return
    if args.profile_leg == "batched":
        print(json.dumps(bench_batched(dc, synth, np, torch, args.batched_images, plain=False, tune=False)))
        return
    if args.profile_leg == "unrolled-plain":
        print(json.dumps(bench_backward(dc, synth, np, torch, only_plain=True)))
        return
    if args.profile_leg == "unrolled":
        print(json.dumps(bench_backward(dc, synth, np, torch, only_fwd_bwd=True)))
        return
    if args.profile_leg == "tensor":
        print(json.dumps(bench_tensor(dc, synth, np, torch)))
        return
    if args.profile_leg == "variants":
        print(json.dumps(bench_variants(dc, synth, np, torch)))
        return
    cfg = synth.CONFIGS["learn"]
    b, d0 = synth.make_inputs(cfg)
    dev = torch.device("cuda:0")
    bt = torch.from_numpy(b).to(dev)
    N, J, K = cfg.n, cfg.j, cfg.k
    H, W = cfg.grid
    D = H * W
    state = {"d": torch.from_numpy(d0).to(dev), "z": None, "theta": None, "gamma": None,
             "mu": torch.ones(K, dtype=torch.float32, device=dev),
             "rho": torch.full((N,), cfg.rho0, dtype=torch.float32, device=dev)}

    def step():
        s = state
        s["z"], s["theta"], _, s["rho"] = dc.code(bt, s["d"], cfg.beta, s["rho"], cfg.t_in, z=s["z"],
                                                  theta=s["theta"], adaptive=True, want_theta=True)
        s["d"], s["mu"], s["gamma"] = dc.learn(bt, s["z"], cfg.fsupp, s["mu"], s["gamma"], cfg.learn_inner,
                                               cfg.learn_cg, out=s["d"])
        s["obj"] = dc.objective(bt, s["d"], s["z"], cfg.beta)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dc.trace_enable(True, every=TRACE_EVERY)
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    dc.trace_enable(False)
    ms_total = evs[0].elapsed_time(evs[-1])
    ms_step = ms_total / args.steps
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    maps_ms, maps_cnt = dc.trace_read(dc.TRACE_CODE_MAPS)
    spec_ms, spec_cnt = dc.trace_read(dc.TRACE_CODE_SPEC)
    la_ms, la_cnt = dc.trace_read(dc.TRACE_LEARN_A)
    lb_ms, lb_cnt = dc.trace_read(dc.TRACE_LEARN_B)
    sr_ms, sr_cnt = dc.trace_read(dc.TRACE_LEARN_SPAN_ROWS)
    sa_ms, sa_cnt = dc.trace_read(dc.TRACE_LEARN_SPAN_APPLY)

    cpit_step = N * K * D * cfg.t_in
    value = cpit_step / (ms_step / 1e3)

    # coding alone (same state, same launch configuration)
    z = state["z"].clone()
    th = state["theta"].clone()
    rho = state["rho"].clone()
    reps = max(3, args.steps)
    dc.code(bt, state["d"], cfg.beta, rho, cfg.t_in, z=z, theta=th, adaptive=True)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(reps):
        dc.code(bt, state["d"], cfg.beta, rho, cfg.t_in, z=z, theta=th, adaptive=True)
    c1.record(stream)
    torch.cuda.synchronize()
    code_ms = c0.elapsed_time(c1) / reps

    fused_avg_ms = maps_ms / max(1, maps_cnt)
    bytes_launch = alg_bytes_per_iter(N, J, K, D)
    achieved = bytes_launch / (fused_avg_ms / 1e3) / 1e9
    flop_launch = (5 * np.log2(D) + 16) * N * K * D
    fused_traffic = counter_traffic("k_fused<128,128,1,0>")

    def hbm_roofline(kernel, alg_bytes, ms_total, count, traffic):
        avg = ms_total / max(1, count)
        ach = alg_bytes / (avg / 1e3) / 1e9 if count else 0.0
        return {"kernel": kernel, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "avg_launch_ms": avg, "launches": count,
                "alg_bytes_per_launch": alg_bytes}

    def alu_roofline(kernel, flops, ms_total, count, traffic):
        avg = ms_total / max(1, count)
        ach = flops / (avg / 1e3) / 1e12 if count else 0.0
        return {"kernel": kernel, "bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_VECTOR_TFLOPS, "traffic": traffic, "avg_launch_ms": avg, "launches": count,
                "flops_per_launch": flops,
                "peak_note": "fp64 vector peak of MI355X (256 CUs x 2.4 GHz x 128 flop/clk); the kernel is "
                             "float64 multiply-adds on LDS-staged operands"}

    roof_fused = {
        "kernel": "k_fused<128,128,1,iter> (back-projection + inverse FFT + soft threshold + forward FFT)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": fused_traffic,
        "avg_launch_ms": fused_avg_ms,
        "launches": maps_cnt,
        "alg_bytes_per_launch": bytes_launch,
        "alu_tflops": flop_launch / (fused_avg_ms / 1e3) / 1e12,
    }
    # per-step time of each candidate for the headline entry: the kernel the
    # step spends most time in
    steps_learn = cfg.learn_inner * (cfg.learn_cg + 1)
    share = {"coding_fused": fused_avg_ms * cfg.t_in}
    extra = {"coding_fused": roof_fused}
    if sa_cnt:
        M1, M2 = cfg.fsupp
        extra["learning_span_apply"] = alu_roofline(
            "l_cc_apply<11, 11> (learning CG step in the span form: filter-space vector times the float64 lag "
            "correlations of the code maps)", span_apply_flops(J, K, M1, M2), sa_ms, sa_cnt,
            counter_traffic("l_cc_apply<11,11>"))
        share["learning_span_apply"] = sa_ms / sa_cnt * steps_learn
        rows_l = 2 * ((M2 + 1) // 2)  # the row kernel's lag slots (even, >= M2)
        extra["learning_span_rows"] = alu_roofline(
            "l_cc_rows<%d> (row stage of the code-map correlation table, once per learning call)" % rows_l,
            span_rows_flops(N, J, K, H, W, M2), sr_ms, sr_cnt, counter_traffic("l_cc_rows<%d>" % rows_l))
        share["learning_span_rows"] = sr_ms / max(1, sr_cnt)
    if la_cnt:
        # the learning passes stream the N K D code spectra, which stay in the
        # Infinity Cache across the step: the HBM peak bounds them from above,
        # a plain copy of such a set is the practical ceiling
        cache_note = ("working set %.1f MB of code spectra, resident in the 256 MB Infinity Cache across the "
                      "step; a plain copy of a set that size reaches ~6.9 TB/s" % (4e-6 * N * K * D))
        extra["learning_pass_a"] = hbm_roofline(
            "l_passA_rows<1> (learning pass A: sum over images of conj(zhat) p, row stage of the support "
            "projection)", alg_bytes_pass_a(N, J, K, H, W, cfg.fsupp[0], cfg.fsupp[1]), la_ms, la_cnt,
            counter_traffic("l_passA_rows<1>"))
        extra["learning_pass_a"]["working_set"] = cache_note
        share["learning_pass_a"] = la_ms / la_cnt * steps_learn
    if lb_cnt:
        extra["learning_pass_b"] = hbm_roofline(
            "l_passB_c<1> (learning pass B: p + sum over filters of zhat U)", alg_bytes_pass_b(N, J, K, H, W),
            lb_ms, lb_cnt, counter_traffic("l_passB_c<1>"))
        share["learning_pass_b"] = lb_ms / lb_cnt * (steps_learn if la_cnt else 1)
    head = max(share, key=share.get)
    roof = dict(extra.pop(head))
    roof["ms_per_step_in_kernel"] = share[head]
    for key in extra:
        extra[key]["ms_per_step_in_kernel"] = share.get(key)

    out = {
        "metric": "ADMM coding iters/sec (N·K·pixels/s) + HBM GB/s; batched & backward vs plain",
        "value": value,
        "unit": "code-pixel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "step_ms_p10_p50_p90": [float(np.percentile(per_step, q)) for q in (10, 50, 90)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "grayscale CSC learning: N=10 images 100x100 padded to 128x128, K=100 filters 11x11, "
                        "beta=1, adaptive rho (rho0=10); step = 10 ADMM coding iterations + learning "
                        "(10 mu x 10 CG) + objective",
            "n": N, "j": J, "k": K, "grid": [H, W], "fsupp": list(cfg.fsupp), "t_in": cfg.t_in,
            "learn_inner": cfg.learn_inner, "learn_cg": cfg.learn_cg,
        },
        "roofline": roof,
        "roofline_kernel": head,
        "roofline_extra": extra,
        "coding_only": {
            "ms_per_call": code_ms,
            "cp_it_per_s": cpit_step / (code_ms / 1e3),
            "alg_gbps": bytes_launch * cfg.t_in / (code_ms / 1e3) / 1e9,
        },
        "traced_avg_launch_ms": {
            "coding_map_kernel": maps_ms / max(1, maps_cnt),
            "coding_spectral": spec_ms / max(1, spec_cnt),
            "learning_pass_a": la_ms / max(1, la_cnt),
            "learning_pass_b": lb_ms / max(1, lb_cnt),
            "learning_span_rows": sr_ms / max(1, sr_cnt),
            "learning_span_apply": sa_ms / max(1, sa_cnt),
        },
        "objective_last": float(state["obj"][-1].item()),
    }

    if not args.no_batched:
        out["batched"] = bench_batched(dc, synth, np, torch, args.batched_images)
    if not args.no_backward:
        out["backward"] = bench_backward(dc, synth, np, torch)
    if not args.no_tensor:
        out["tensor"] = bench_tensor(dc, synth, np, torch)
    if not args.no_variants:
        out["variants"] = bench_variants(dc, synth, np, torch)

    if not args.no_cpu_baseline:
        import oracle
        n_cpu = max(1, min(args.cpu_images, N))
        bs = b[:n_cpu]
        t0 = time.perf_counter()
        o = oracle.code(bs, d0, cfg.beta, cfg.rho0, cfg.t_in, adaptive=True)
        oracle.learn(bs, o["z"], cfg.fsupp, np.ones(K), None, cfg.learn_inner, cfg.learn_cg)
        oracle.objective(bs, d0, o["z"], cfg.beta)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": n_cpu * K * D * cfg.t_in / t_cpu,
            "unit": "code-pixel-iterations/s",
            "cores": 1,
            "kind": "oracle",
            "sample": "first %d of the 10 images, one outer step (10 ADMM iterations + learning 10x10 + "
                      "objective), numpy float64, single thread; %.1f s" % (n_cpu, t_cpu),
            "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
        }
        # all cores: the coding half of the step, images in parallel, in a
        # child process (it forks workers; this process has initialised the GPU)
        import subprocess
        procs = max(1, min(16, os.cpu_count() or 1, N))
        try:
            res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-all-cores", str(procs)],
                                 capture_output=True, text=True, timeout=300)
            allc = json.loads(res.stdout.strip().splitlines()[-1])
            out["cpu_baseline"]["all_cores_coding"] = {
                "value": allc["value"], "unit": "code-pixel-iterations/s", "cores": procs,
                "sample": "oracle coding of all 10 images (10 adaptive ADMM iterations each), one image per "
                          "worker process; %.1f s" % allc["seconds"],
            }
        except (subprocess.SubprocessError, ValueError, KeyError, IndexError) as exc:
            out["cpu_baseline"]["all_cores_coding"] = {"error": str(exc)[:200]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
