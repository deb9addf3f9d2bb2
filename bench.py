#!/usr/bin/env python3
"""NLL + gradient evaluations per second at 1M events x 20 waves on one MI355X.

Workload (the fit-iteration hot path of Eq. 3 in arXiv:1108.5673): 1,000,000
synthetic J/psi -> gamma K+K- shaped data events, 20 waves (10 Breit-Wigner
masses in 1.0-2.6 GeV x J in {0, 2}), MC normalisation from 2M accepted of 4M
generated flat events, and 200 parameter points along a seeded random walk
starting at the generating point.  One step = one pwa_nll_grad call: the NLL and
its 40-component gradient for one parameter point, V in and results out through
host memory, with the table already resident in HBM.

Timed paths: the fused one-pass kernel over the packed complex64 table (the
reported value), the plain two-pass FP64 table kernels (the baseline), and the
fused kernel over a complex128 table (ablation).  The main kernel's device time
is taken inside the timed region with two HIP events per launch, on the stream
the kernel runs on, which the runtime stamps with the dispatch's own begin and
end; it is turned into achieved bandwidth from the algorithmic bytes (1600 B per
event: the 190 off-diagonal complex64 entries of the Hermitian table and its 20
real diagonal entries).  Per-call latency percentiles are host wall-clock times of the
synchronous call.  The CPU
oracle is timed on a bounded sample of the same walk on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "table_fused_w20_n1m_traffic.json")


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    from paper_1108_5673_amd.profiling import kernel_source_hash
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_model(model, points, steps, warmup):
    import torch
    for k in range(warmup):
        model.nll_grad(points[k % len(points)])
    torch.cuda.synchronize()
    # kernel time from HIP events on every 32nd evaluation of the timed region
    # (a stamped launch costs its call about 18 us; one in 32 adds less than
    # 1 us to the average step)
    model.set_timing(True, every=32)
    model.timing()
    results, lat = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        a = time.perf_counter()
        results.append(model.nll_grad(points[k % len(points)]))
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms, launches = model.timing()
    model.set_timing(False)
    q = np.percentile(np.array(lat) * 1e6, [10, 50, 90])
    return {
        "seconds": t1 - t0,
        "evals_per_s": steps / (t1 - t0),
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "kernel_ms": kernel_ms / max(1, launches),
        "latency_us": {"p10": q[0], "p50": q[1], "p90": q[2]},
        "results": results,
    }


def host_cpu():
    """CPU model (from /proc/cpuinfo), logical CPUs this process may use and
    logical CPUs of the machine."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count()}


def mfma_flops(n_events, n_waves, k, v_parts, bf16=False):
    """Matrix-core FLOPs of one batched pass as the kernel issues them: per
    16-event tile (32 rows) and 32 vectors, the forward product (16-wide KD
    steps x V parts, 32x32x16 MFMAs of 32768 FLOP; one step fewer for bf16
    when 2W mod 16 is 1..8) and the adjoint (per full
    32-row block 2 slot steps x 2 weight parts of the same MFMA; a last block
    of 16 rows as 2 vector blocks x 2 weight parts of the 16x16x32 MFMA,
    16384 FLOP each)."""
    kd = (2 * n_waves + 15) // 16 * 16
    rf, rem = (kd // 16) // 2, (kd // 16) % 2
    tiles = (n_events + 15) // 16
    col_blocks = (k + 31) // 32
    fwd = (kd // 16) * v_parts
    if bf16 and 0 < (2 * n_waves) % 16 <= 8:
        fwd -= 1   # the second part's last K-step rides in the first part's padding
    per = (fwd + rf * 2 * 2) * 32768 + rem * 2 * 2 * 16384
    return tiles * col_blocks * per


def mfma_algorithmic_flops(n_events, n_waves, k, v_parts):
    """The products the batched pass must form, without padding: the forward
    S = A V as a real product of 2N rows x 2W x 2K per V part (8 N W K FLOP
    each) and the adjoint over two weight parts (8 N W K each)."""
    return 8 * n_events * n_waves * k * (v_parts + 2)


def bench_batched(args):
    """The 256 random starting points of w20_n1m_k256 in one pass of the
    matrix-core amplitude forms (bf16 and fp16 amplitudes)."""
    import torch
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth
    s = synth.make_sample("w20_n1m_k256")
    d32, mc32 = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    out = {"workload": "w20_n1m_k256: 1M events x 20 waves, K = 256 vectors Re, Im ~ N(0, 1), "
                       "amplitude form on the matrix cores", "K": 256}
    ref = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.get()
        M64 = o.mc_matrix(s.mc, s.n_gen)
        t = time.perf_counter()
        ref = {j: o.nll_amp(s.data, M64, s.points[j]) for j in (0, 85, 170, 255)}
        out["oracle"] = {"evals_per_s": len(ref) / (time.perf_counter() - t),
                         "cores": o.num_threads(),
                         "sample": "vectors 0, 85, 170, 255 on the FP64 amplitudes"}
    for form, parts in (("amplitude_bf16", 2), ("amplitude_fp16", 2)):
        m = pwa.Model(d32, mc32, s.n_gen, form=form)
        # the matrix-core kernel takes some tens of passes to reach its steady
        # speed on a box (its time falls by about 15 % over the first 40)
        for _ in range(40):
            pwa.nll_batched([m], [s.points])
        torch.cuda.synchronize()
        # kernel time from event stamps on every 8th pass (a stamped launch
        # costs about 18 us of the call)
        m.set_timing(True, every=8)
        m.timing()
        reps = 48
        t = time.perf_counter()
        for _ in range(reps):
            [(nll, g)] = pwa.nll_batched([m], [s.points])
        dt = (time.perf_counter() - t) / reps
        ms, n = m.timing()
        kus = 1e3 * ms / max(1, n)
        fl = mfma_flops(s.data.shape[0], 20, 256, parts, bf16=(form == "amplitude_bf16"))
        fa = mfma_algorithmic_flops(s.data.shape[0], 20, 256, parts)
        r = {"evals_per_s": 256 / dt, "batch_us": 1e6 * dt, "kernel_us": kus,
             "mfma_tflops": fa / (kus * 1e-6) / 1e12, "mfma_peak_tflops": 2500.0,
             "mfma_frac": fa / (kus * 1e-6) / 2.5e15,
             "mfma_flops_algorithmic": fa, "mfma_flops_issued": fl,
             "mfma_issued_tflops": fl / (kus * 1e-6) / 1e12,
             "mfma_issued_frac": fl / (kus * 1e-6) / 2.5e15,
             "events_iter_per_s": 256 / dt * s.data.shape[0]}
        if ref is not None:
            r["max_abs_dnll_vs_fp64_amplitudes"] = max(abs(nll[j] - ref[j][0]) for j in ref)
            r["max_rel_grad_vs_fp64_amplitudes"] = max(
                float(np.linalg.norm(g[j] - ref[j][1]) / np.linalg.norm(ref[j][1])) for j in ref)
            # the kernel's own error: the oracle on the identical stored 16-bit
            # amplitudes (the model's copy, widened exactly)
            a16 = m.table().astype(np.complex128)
            M32 = o.mc_matrix(mc32.astype(np.complex128), s.n_gen)
            same = {j: o.nll_amp(a16, M32, s.points[j]) for j in ref}
            del a16
            r["max_abs_dnll_vs_identical_inputs"] = max(abs(nll[j] - same[j][0]) for j in same)
            r["max_rel_dnll_vs_identical_inputs"] = max(
                abs(nll[j] - same[j][0]) / abs(same[j][0]) for j in same)
            r["max_rel_grad_vs_identical_inputs"] = max(
                float(np.linalg.norm(g[j] - same[j][1]) / np.linalg.norm(same[j][1]))
                for j in same)
        out[form] = r
        log("batched %s: %.0f evals/s, kernel %.1f us (%.0f TFLOP/s algorithmic, %.0f issued on "
            "the matrix cores)" % (form, r["evals_per_s"], kus, r["mfma_tflops"],
                                   r["mfma_issued_tflops"]))
        m.close()
    return out


def bench_amplitude(args):
    """The FP32 amplitude form at 2M events x 32 waves, 4M accepted MC (the
    differentiation workload's sizes; flat synthetic amplitudes drawn on the
    device): NLL+gradient throughput in the default storage shape and in the
    shape pwa_tune_amplitude_shape picks."""
    import torch
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth
    W, N = 32, 2_000_000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11085673 + 3)
    ws = synth.wave_set(W)
    d = synth._amplitudes_torch(N, ws, gen, "cuda")
    mc = synth._amplitudes_torch(2 * N, ws, gen, "cuda")
    m = pwa.Model(d, mc, 4 * N, form="amplitude")
    d_host = mc_host = None
    if not args.no_cpu_baseline:
        d_host, mc_host = d.cpu().numpy(), mc.cpu().numpy()
    del d, mc
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 32, 1])))
    pts = [synth.random_v(rng, W) for _ in range(20)]
    out = {"workload": "amplitude form, 2M events x 32 waves (512 MB complex64), 4M accepted MC; "
                       "flat synthetic amplitudes; 20 random V (Re, Im ~ N(0, 1))"}
    ref = None
    if not args.no_cpu_baseline:
        # the oracle on the same complex64 amplitudes (widened), its own M
        import oracle
        o = oracle.get()
        d_h = d_host.astype(np.complex128)
        M64 = o.mc_matrix(mc_host.astype(np.complex128), 4 * N)
        t = time.perf_counter()
        ref = {j: o.nll_amp(d_h, M64, pts[j]) for j in (0, 1)}
        out["oracle"] = {"evals_per_s": len(ref) / (time.perf_counter() - t),
                         "cores": o.num_threads(), "sample": "points 0 and 1, all 2M events"}
        del d_h
    for tag in ("default", "tuned"):
        if tag == "tuned":
            m.tune_amplitude_shape(5)
        r = time_model(m, pts, args.steps, args.warmup)
        kus = 1e3 * r["kernel_ms"]
        out[tag] = {"shape": list(m.amplitude_shape()), "evals_per_s": r["evals_per_s"],
                    "kernel_us": kus, "achieved_gbs": 8.0 * W * N / (kus * 1e-6) / 1e9,
                    "frac_of_8tbs": 8.0 * W * N / (kus * 1e-6) / 8e12}
        if ref is not None:
            res = r["results"]
            out[tag]["max_rel_dnll"] = max(abs(res[j][0] - ref[j][0]) / abs(ref[j][0]) for j in ref)
            out[tag]["max_rel_grad"] = max(float(np.linalg.norm(res[j][1] - ref[j][1]) /
                                                 np.linalg.norm(ref[j][1])) for j in ref)
        log("amplitude w32 n2m (%s shape %s): %.0f evals/s, kernel %.1f us (%.0f GB/s)"
            % (tag, out[tag]["shape"], r["evals_per_s"], kus, out[tag]["achieved_gbs"]))
    # achievable read bandwidth on the same stored amplitudes (a plain
    # non-temporal reader over every stored byte, pwa_read_ceiling)
    rc = m.read_ceiling(10)
    out["read_ceiling_gbs"] = rc["gbs"]
    out["read_ceiling_bytes"] = rc["bytes"]
    for tag in ("default", "tuned"):
        out[tag]["frac_of_read_ceiling"] = out[tag]["achieved_gbs"] / rc["gbs"]
    log("amplitude w32 n2m: plain read of the stored %.0f MB: %.1f us, %.0f GB/s"
        % (rc["bytes"] / 1e6, 1e3 * rc["ms"], rc["gbs"]))
    m.close()
    return out


def bench_multi(args):
    """64 amplitude-form models of uneven size (W uniform in 8..48, N log-uniform
    in 1e5..4e6, 2N accepted MC each), one NLL+gradient of every model per
    iteration through one pwa_nll_batched call (per class of storage shape one
    amplitude launch, then one assembly, replayed from a captured graph), 500
    iterations along a random walk per model, called through pwa.Batch; and
    the same iterations through the list form and as 64 separate calls."""
    import torch
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth
    sizes = synth.uneven_sizes()
    t = time.perf_counter()
    models, keep, v0 = [], {}, []
    small = sorted(range(len(sizes)), key=lambda i: sizes[i][1])[:2]
    for i, um in enumerate(synth.uneven_models(sizes)):
        models.append(pwa.Model(um.data, um.mc, 2 * um.n_acc, form="amplitude"))
        if i in small and not args.no_cpu_baseline:
            keep[i] = (um.data.cpu().numpy(), um.mc.cpu().numpy(), 2 * um.n_acc)
        v0.append(um.v0)
        del um
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("built 64 uneven models in %.1f s" % (time.perf_counter() - t))
    # storage shape per model, chosen by timing (pwa_tune_amplitude_shape)
    t = time.perf_counter()
    shapes = {}
    for m in models:
        sh = "%dx%d" % m.tune_amplitude_shape(5)
        shapes[sh] = shapes.get(sh, 0) + 1
    tune_s = time.perf_counter() - t
    log("tuned the storage shapes in %.1f s: %s" % (tune_s, shapes))
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 64, 2])))
    iters = 500
    walk = []
    cur = [v.copy() for v in v0]
    for _ in range(iters):
        cur = [c + 0.01 * (rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape))
               for c in cur]
        walk.append(cur)
    # one pwa_nll_batched call per iteration through pwa.Batch (handles, counts
    # and output buffers set up once; one flat parameter array per iteration)
    batch = pwa.Batch(models)
    flat = [np.concatenate([np.ascontiguousarray(w, np.complex128).view(np.float64)
                            for w in walk[k]]) for k in range(iters)]
    for k in range(5):
        batch(flat[k])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(iters):
        res = batch(flat[k])
    dt = (time.perf_counter() - t) / iters
    # the same call through the list form (nll_batched converts 64 arrays a call)
    list_iters = 50
    t = time.perf_counter()
    for k in range(list_iters):
        pwa.nll_batched(models, [w[None, :] for w in walk[k]])
    dt_list = (time.perf_counter() - t) / list_iters
    seq_iters = 50
    t = time.perf_counter()
    for k in range(seq_iters):
        for m, w in zip(models, walk[k]):
            m.nll_grad(w)
    dt_seq = (time.perf_counter() - t) / seq_iters
    n_tot = sum(n for w, n in sizes)
    bytes_it = sum(m.info()["stream_bytes"] for m in models)
    out = {"workload": "64 models: W uniform 8..48, N log-uniform 1e5..4e6 (%d events in all), "
                       "2N accepted MC each, flat synthetic amplitudes; 500 iterations" % n_tot,
           "iteration_ms": 1e3 * dt, "evals_per_s": 64 / dt,
           "events_iter_per_s": n_tot / dt, "achieved_gbs": bytes_it / dt / 1e9,
           "frac_of_8tbs": bytes_it / dt / 8e12, "separate_calls_iteration_ms": 1e3 * dt_seq,
           "list_api_iteration_ms": 1e3 * dt_list,
           "tuned_shapes": shapes, "tuning_s": tune_s,
           "speedup_vs_separate_calls": dt_seq / dt}
    if keep:
        import oracle
        o = oracle.get()
        last = walk[iters - 1]
        worst_n, worst_g = 0.0, 0.0
        t_or, ev_or = 0.0, 0
        for i, (d, mc, n_gen) in keep.items():
            M = o.mc_matrix(mc.astype(np.complex128), n_gen)
            d128 = d.astype(np.complex128)
            t = time.perf_counter()
            rn, rg, _ = o.nll_amp(d128, M, last[i])
            t_or += time.perf_counter() - t
            ev_or += d.shape[0]
            nll, g = res[i][0][0], res[i][1][0]
            dn = abs(nll - rn) / max(1.0, abs(rn))
            dg = float(np.linalg.norm(g - rg) / np.linalg.norm(rg))
            worst_n = max(worst_n, dn if np.isfinite(dn) else np.inf)
            worst_g = max(worst_g, dg if np.isfinite(dg) else np.inf)
        out["parity"] = {"models": sorted(keep), "max_rel_dnll": worst_n, "max_rel_grad": worst_g,
                         "reference": "oracle on the same complex64 amplitudes"}
        out["oracle"] = {"events_iter_per_s": ev_or / t_or, "cores": o.num_threads(),
                         "sample": "one evaluation of each of the two smallest models"}
    log("multi-model: %.2f ms per iteration of 64 models (%.0f GB/s); list form %.2f ms; "
        "separate calls %.2f ms" % (1e3 * dt, bytes_it / dt / 1e9, 1e3 * dt_list, 1e3 * dt_seq))
    for m in models:
        m.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-baselines", action="store_true", help="time only the fused kernel")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-vector matrix-core measurement")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the 64-model batch measurement")
    ap.add_argument("--no-amplitude", action="store_true",
                    help="skip the amplitude-form measurement at 2M events x 32 waves")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the likelihood hot path is built and timed on a "
              "single MI355X; multi-GPU runs are not part of this build (got --gpus %d, "
              "WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.init()
    torch.cuda.set_device(0)

    t = time.perf_counter()
    sample = synth.make_sample("w20_n1m")
    log("generated w20_n1m in %.1f s" % (time.perf_counter() - t))
    pts = sample.points
    d32 = sample.data.astype(np.complex64)
    mc32 = sample.mc.astype(np.complex64)

    t = time.perf_counter()
    fused = pwa.Model(d32, mc32, sample.n_gen, form="table")
    torch.cuda.synchronize()
    log("built fused complex64 table in %.2f s" % (time.perf_counter() - t))
    info = fused.info()
    prefit = fused.build_timing()
    log("build steps on the device: table %.2f ms, MC integral %.2f ms"
        % (prefit["table_ms"], prefit["mc_ms"]))
    f = time_model(fused, pts, args.steps, args.warmup)
    log("fused: %.1f evals/s, kernel %.1f us, grid %d blocks on %d CUs"
        % (f["evals_per_s"], 1e3 * f["kernel_ms"], info["grid_blocks"], info["compute_units"]))
    # the achievable read bandwidth on the same stored bytes: the fused
    # kernel's loads with its arithmetic taken out
    ceiling = fused.read_ceiling(reps=10)
    log("the kernel's loads alone on the same %.2f GB: %.1f us, %.0f GB/s"
        % (ceiling["bytes"] / 1e9, 1e3 * ceiling["ms"], ceiling["gbs"]))

    # a full fit on the same model from a random start (L-BFGS in the library,
    # one pwa_nll_grad per objective call)
    from paper_1108_5673_amd import fit as pwa_fit
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 20, 1])))
    v0 = synth.random_v(rng, 20)
    t = time.perf_counter()
    v_fit, fres = pwa_fit.fit_lbfgs(fused, v0)
    fit_s = time.perf_counter() - t
    fit_info = {"start": "Re, Im V ~ N(0, 1) (the FUMILI driver scales it to mu = N)",
                "status": fres["message"],
                "iterations": fres["iterations"], "evaluations": fres["evaluations"],
                "seconds": fit_s, "evals_per_s": fres["evaluations"] / fit_s,
                "nll": fres["f"], "grad_norm": fres["grad_norm"]}
    log("fit from a random start: %s after %d iterations, %d evaluations, %.3f s"
        % (fres["message"], fres["iterations"], fres["evaluations"], fit_s))
    # the same start with FUMILI steps (NLL and gradient at trial points, the
    # FUMILI matrix at the points taken) on the amplitude form of the same
    # sample; then both drivers from a start near the generating point (5 %
    # complex noise per wave), the regime of fits repeated around a solution
    amp = pwa.Model(d32, mc32, sample.n_gen, form="amplitude")
    t = time.perf_counter()
    v_fu, fu = pwa_fit.fit_fumili(amp, v0)
    fu_s = time.perf_counter() - t
    fit_info["fumili"] = {"status": fu["message"], "iterations": fu["iterations"],
                          "evaluations": fu["evaluations"], "seconds": fu_s, "nll": fu["f"],
                          "grad_norm": fu["grad_norm"], "form": "amplitude (complex64)"}
    log("FUMILI fit from the same start: %s after %d iterations, %.3f s"
        % (fu["message"], fu["iterations"], fu_s))
    v_near = sample.v_true * (1 + 0.05 * (rng.standard_normal(20) + 1j * rng.standard_normal(20)))
    near = {"start": "V_true (1 + 0.05 (xi + i eta)), xi, eta ~ N(0, 1) per wave"}
    for tag, fn, mdl in (("fumili", pwa_fit.fit_fumili, amp), ("lbfgs", pwa_fit.fit_lbfgs, fused)):
        t = time.perf_counter()
        _, r = fn(mdl, v_near)
        near[tag] = {"status": r["message"], "iterations": r["iterations"],
                     "evaluations": r["evaluations"], "seconds": time.perf_counter() - t,
                     "nll": r["f"]}
    fit_info["near_generating_point"] = near
    log("from a start near the generating point: FUMILI %d iterations, L-BFGS %d"
        % (near["fumili"]["iterations"], near["lbfgs"]["iterations"]))
    # one NLL + gradient + FUMILI matrix call at the start point, and the
    # oracle's matrix on the same stored amplitudes beside it
    for _ in range(3):
        amp.nll_grad_hess(v0)
    reps = 20
    t = time.perf_counter()
    for _ in range(reps):
        _, _, h_gpu = amp.nll_grad_hess(v0)
    call_s = (time.perf_counter() - t) / reps
    fm = {"call_us": 1e6 * call_s, "sample": "V = the fit's start, all 1M events, W = 20"}
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.get()
        t = time.perf_counter()
        h_or, _ = o.fumili_amp(d32.astype(np.complex128), v0)
        fm["oracle_s"] = time.perf_counter() - t
        fm["oracle_cores"] = o.num_threads()
        fm["rel_frobenius_vs_oracle"] = float(np.linalg.norm(h_gpu - h_or) / np.linalg.norm(h_or))
    fit_info["fumili_matrix"] = fm
    log("NLL + gradient + FUMILI matrix: %.1f us per call%s"
        % (fm["call_us"], "" if "oracle_s" not in fm else
           "; oracle matrix %.2f s on %d threads, rel. difference %.1e"
           % (fm["oracle_s"], fm["oracle_cores"], fm["rel_frobenius_vs_oracle"])))
    amp.close()

    out = {}
    if not args.no_baselines:
        plain = pwa.Model(sample.data, sample.mc, sample.n_gen, form="table_fp64_plain")
        p = time_model(plain, pts, args.steps, args.warmup)
        log("plain fp64: %.1f evals/s, kernels %.1f us" % (p["evals_per_s"], 1e3 * p["kernel_ms"]))
        plain_info = plain.info()
        plain.close()
        f64 = pwa.Model(sample.data, sample.mc, sample.n_gen, form="table_fp64")
        q = time_model(f64, pts, args.steps, args.warmup)
        log("fused fp64: %.1f evals/s, kernel %.1f us" % (q["evals_per_s"], 1e3 * q["kernel_ms"]))
        f64_info = f64.info()
        f64.close()
        out["plain_fp64_table"] = {
            "value": p["evals_per_s"], "ms_per_step": p["ms_per_step"],
            "kernel_us": 1e3 * p["kernel_ms"],
            "achieved_gbs": plain_info["stream_bytes"] / (p["kernel_ms"] * 1e-3) / 1e9,
        }
        out["fused_fp64_table"] = {
            "value": q["evals_per_s"], "ms_per_step": q["ms_per_step"],
            "kernel_us": 1e3 * q["kernel_ms"],
            "achieved_gbs": f64_info["stream_bytes"] / (q["kernel_ms"] * 1e-3) / 1e9,
        }
        out["speedup_vs_plain_fp64"] = f["evals_per_s"] / p["evals_per_s"]

    batched = None
    if not args.no_batched:
        batched = bench_batched(args)
    amplitude = None
    if not args.no_amplitude:
        amplitude = bench_amplitude(args)
    multi = None
    if not args.no_multi:
        multi = bench_multi(args)

    achieved = info["stream_bytes"] / (f["kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                "kernel": "k_table_fused (complex64 table)", "kernel_us": 1e3 * f["kernel_ms"],
                "bytes_per_launch": info["stream_bytes"], "grid_blocks": info["grid_blocks"],
                "read_ceiling_gbs": ceiling["gbs"], "frac_of_read_ceiling": achieved / ceiling["gbs"],
                "read_ceiling": "fastest of 10 passes of the fused kernel's loads (same grid, "
                                "shape and order) with its arithmetic taken out, on the same "
                                "stored table (pwa_read_ceiling)"}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.get()
        t = time.perf_counter()
        T = o.table(d32.astype(np.complex128)).astype(np.complex64).astype(np.complex128)
        prefit["oracle_table_s"] = time.perf_counter() - t
        t = time.perf_counter()
        M = o.mc_matrix(mc32.astype(np.complex128), sample.n_gen)
        prefit["oracle_mc_s"] = time.perf_counter() - t
        log("oracle table %.2f s, MC matrix %.2f s"
            % (prefit["oracle_table_s"], prefit["oracle_mc_s"]))
        times, k, dn, dg = [], 0, [], []
        while k < min(len(pts), args.steps) and (k < 2 or sum(times) < args.cpu_seconds):
            t = time.perf_counter()
            rn, rg, _ = o.nll_table(T, M, pts[k])
            times.append(time.perf_counter() - t)
            gn, gg = f["results"][k]
            dn.append(abs(gn - rn))
            dg.append(float(np.linalg.norm(gg - rg) / np.linalg.norm(rg)))
            k += 1
        cpu = {"value": k / sum(times), "unit": "NLL+grad evals/s", "cores": o.num_threads(),
               "kind": "oracle",
               "sample": "first %d of the 200 walk points, all 1M events, FP64 table form "
                         "(packed complex64 table widened to complex128)" % k}
        # the same evaluation on one host thread (first walk point), and the host
        n_thr = o.num_threads()
        o.set_num_threads(1)
        t = time.perf_counter()
        o.nll_table(T, M, pts[0])
        cpu["one_thread"] = {"value": 1.0 / (time.perf_counter() - t), "cores": 1,
                             "sample": "walk point 0"}
        o.set_num_threads(n_thr)
        cpu["host"] = host_cpu()
        parity = {"points": k, "max_abs_dnll": max(dn), "max_rel_grad_err": max(dg),
                  "reference": "oracle on the identical stored complex64 table"}
        del T
        log("oracle: %.3f evals/s on %d threads (%.3f on one); max |dNLL| %.2e, max grad rel %.2e"
            % (cpu["value"], cpu["cores"], cpu["one_thread"]["value"], max(dn), max(dg)))

    line = {
        "metric": "NLL+grad evals/s at 1M events, 20 waves: fused FP32 vs plain FP64 table",
        "value": f["evals_per_s"],
        "unit": "NLL+grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "complex64 packed table (FP64 arithmetic and accumulation)",
        "data": "synthetic",
        "config": {"workload": "w20_n1m: 1M events x 20 waves, packed complex64 table "
                               "(190 complex off-diagonal + 20 real diagonal entries, 1600 B per event), "
                               "MC 2M accepted of 4M "
                               "generated, 200-point random walk from the generating point",
                   "n_events": sample.data.shape[0], "n_waves": 20, "n_mc_acc": sample.mc.shape[0],
                   "n_mc_gen": sample.n_gen, "points": len(pts)},
        "events_iter_per_s": f["evals_per_s"] * sample.data.shape[0],
        "latency_us": f["latency_us"],
        "prefit": prefit,
        "fit": fit_info,
        "amplitude_w32_n2m": amplitude,
        "batched_k256": batched,
        "multi_model_64": multi,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
