#!/usr/bin/env python3
"""Benchmark of the chi^2 hot path on one MI355X.

Workload: chi2Profile at Nxy = 2048, M = 10^6 uv points, FP64 -- a radial
profile of Nr = 4096 samples (gapped power law) swept into a 2048^2 image at
dxy = 0.003'', uv points log-uniform over ALMA C43-10 baselines at 1.3 mm,
inc = 45 deg, PA = 120 deg, Vobs = model + N(0, 1e-3^2) noise, w = 1e6.
The observations are registered once as a device-resident dataset (inputs
resident in HBM before the timed region).

A step is one batched evaluation of K models (the walkers of an ensemble
sampler: perturbed profiles and geometry) through the whole path -- sweep +
row FFT, column FFT, sample + phase + chi^2, reduction -- replayed from a HIP
graph; `value` counts chi^2 evaluations per second.  The plain form (one
call per evaluation) is measured on the same dataset and reported beside it
with its p50/p99 latency.

Prints one JSON line.  Per-kernel times come from the dispatch timestamps
recorded on the launch stream inside the library (a separate pass over the
same steps); the roofline entry is for the kernel with the largest share of
the batched step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic__chi2Profile_2048_M1e6_K64.md")
METRIC = "χ² evals/s at 2048², 1M uv (FP64), batched/served vs plain; p50/p99 latency"


def progress(what):
    """One line on stderr per section (the JSON result goes to stdout)."""
    print(f"bench: {what}", file=sys.stderr, flush=True)


def _ensure_built():
    from paper_1709_06999_amd import _native

    if not os.path.exists(_native.LIB_PATH):
        from paper_1709_06999_amd.build import build_library

        build_library()


def algorithmic_bytes(N, Nr, M, Q, P, kind="profile", p=8):
    """Bytes each kernel must move at least once (inputs, outputs, the one
    round trip of the row -> column intermediate), for the part of the half
    spectrum the points reach: columns [0, Q), rows [-P, P].

    profile: the swept image is even in both axes, so its spectrum is real:
      rows [0, N/2] -> real intermediate (N/2+1) x Qe, real spectrum
      (P+1) x Qe (Qe = Q rounded up to even);
    image: general real image -> complex intermediate N x Q, complex
      spectrum (2P+1) x Q."""
    red = 8 * ((M + 1023) // 1024) + 8
    if kind == "profile":
        Qe = Q + (Q & 1)
        inter = (N // 2 + 1) * Qe * p
        spec = (P + 1) * Qe * p
        return {"k_rows_sym": Nr * p + inter, "k_rows_even": Nr * p + inter, "k_cols_sym": inter + spec,
                "k_cols_even": inter + spec, "k_sample_sym_chi2": 5 * p * M + spec, "k_reduce": red}
    inter = N * Q * 2 * p
    spec = Q * (2 * P + 1) * 2 * p
    return {"k_rows_image": N * N * p + inter, "k_cols": inter + spec,
            "k_sample_chi2": 5 * p * M + spec, "k_reduce": red}


def path_bytes(N, Nr, M, p=8):
    """Bytes of one chi2Profile evaluation as the roofline of the whole path
    counts them: the profile, the full half spectrum written and read once
    as the row -> column intermediate and once as the spectrum, and five
    observation columns; with the gradient also the residuals, a second pass
    over the observations, the scatter grid and the transposed transforms
    (4 half-spectrum passes) and the profile gradient."""
    H = N * (N // 2 + 1)
    chi2 = p * Nr + 2 * (2 * p * H) + 5 * p * M
    return {"chi2": chi2, "chi2_grad": chi2 + 2 * p * M + 5 * p * M + 4 * (2 * p * H) + p * Nr}


# algorithmic FP64 operations per unit (FMA = 2, sin / cos / sqrt = 1 each)
SWEEP_FLOPS_PER_PIXEL = 13   # x, y 2, x / cos(inc) 1, rho^2 2, sqrt 1, t 2, fraction 1, lerp 3, area 1
SAMPLE_FLOPS_PER_POINT = 35  # per profile job and uv point: rotation 6, grid scale 2, fractions
                             # 2, bilinear 11, phase argument 3, sin + cos 2, V 2, chi^2 term 7


def fft_flops(N, Q, K=1):
    """Algorithmic flops of the two FFT passes of the profile path for K jobs.
    Row pass: the sweep of the quarter image ((N/2+1)^2 pixels) and, per pair
    of (even) rows, a complex FFT of length N/2 at 5 L log2 L plus 12 flops per
    point of pre- and post-processing -- the half-length transform, whichever
    variant runs (the full-length one does redundant work).  Column pass:
    columns [0, Qe) two at a time, complex FFT of length N, whichever variant
    runs (the half-length one, kb_cols_even, does less)."""
    Qe = Q + (Q & 1)
    h = N // 2
    rows = (N // 4 + 1) * (5.0 * h * math.log2(h) + 12.0 * h) + (h + 1) ** 2 * SWEEP_FLOPS_PER_PIXEL
    cols = (Qe // 2) * 5.0 * N * math.log2(N)
    return {"kb_rows_sym": K * rows, "kb_rows_even": K * rows, "kb_cols_sym": K * cols,
            "kb_cols_even": K * cols}


def sample_flops(M, K=1):
    """Algorithmic flops of the sampling pass: K profile jobs at M points."""
    return {"kb_sample_sym_chi2": float(K) * M * SAMPLE_FLOPS_PER_POINT}


SAMPLE_IMG_FLOPS_PER_POINT = 48  # per image job and point: rotation + deprojection 7, fractions
                                 # 2, weights 5, complex bilinear 14, mirror and flux 2, phase
                                 # argument 3, sin + cos 2, V 6, chi^2 term 7
RIDGE = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)   # flop per byte


def image_alg(N, M, Q, P, p=8):
    """Algorithmic bytes and flops of the three kernels of one chi2Image on a
    dataset (columns [0, Q), rows [-P, P] of the complex half spectrum).  Row
    pass: each real row of length N as a complex FFT of length N/2 (5 L log2 L)
    and the split into Q outputs (12 flops each); column pass: Q complex FFTs
    of length N."""
    inter = N * Q * 2 * p
    spec = Q * (2 * P + 1) * 2 * p
    h = N // 2
    lg = 5.0 * N * math.log2(N)
    ab = {"k_rows_image": N * N * p + inter, "k_cols": inter + spec,
          "k_sample_chi2": 5 * p * M + spec, "k_reduce": 8 * ((M + 1023) // 1024) + 8,
          # gradient: the scatter grid written once, transposed passes (columns:
          # grid -> N x Q intermediate; rows: intermediate -> N^2 gradient)
          "k_sample_scatter": 5 * p * M + 2 * spec, "k_adj_cols": spec + inter,
          "k_adj_rows": inter + N * N * p}
    fl = {"k_rows_image": N * (5.0 * h * math.log2(h) + 12.0 * Q), "k_cols": Q * lg,
          "k_sample_chi2": float(M) * SAMPLE_IMG_FLOPS_PER_POINT,
          "k_sample_scatter": float(M) * (SAMPLE_IMG_FLOPS_PER_POINT + 24),
          "k_adj_cols": Q * lg, "k_adj_rows": (N // 2) * lg}
    return ab, fl


def kernel_roofline(kern, alg_bytes, alg_flops):
    """Annotate per-kernel times with algorithmic GB/s and TFLOP/s and return
    the roofline of the kernel with the largest share of the time: bound by
    HBM when its arithmetic intensity is below the FP64 ridge, else by the
    FP64 vector ALUs."""
    for k, x in kern.items():
        t = x["avg_us"] * 1e-6
        if k in alg_bytes:
            x["alg_bytes"] = alg_bytes[k]
            x["alg_GBps"] = alg_bytes[k] / t / 1e9
        if k in alg_flops:
            x["alg_flops"] = alg_flops[k]
            x["alg_TFLOPs"] = alg_flops[k] / t / 1e12
    dom = max((k for k in kern if k in alg_bytes), key=lambda k: kern[k]["avg_us"])
    x = kern[dom]
    fl = alg_flops.get(dom, 0.0)
    if fl / alg_bytes[dom] >= RIDGE:
        r = {"bound": "alu", "kernel": dom, "achieved": round(x["alg_TFLOPs"], 3),
             "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": round(x["alg_TFLOPs"] / FP64_PEAK_TFLOPS, 4)}
    else:
        r = {"bound": "hbm", "kernel": dom, "achieved": round(x["alg_GBps"], 1),
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(x["alg_GBps"] / HBM_PEAK_GBS, 4)}
    r.update({"alg_bytes_per_launch": alg_bytes[dom], "alg_flops_per_launch": fl,
              "avg_us": round(x["avg_us"], 3)})
    return r


def source_digest():
    """SHA-256 over the HIP sources (file names and code, sorted), comments and
    blank lines left out: ties stored counter readings to the kernels they
    were taken from, whatever their comments say."""
    import hashlib
    import re

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1709_06999_amd", "csrc")
    for name in sorted(os.listdir(d)):
        h.update(name.encode())
        with open(os.path.join(d, name), encoding="utf-8") as f:
            code = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        code = "\n".join(ln.rstrip() for ln in (re.sub(r"//.*", "", x) for x in code.splitlines())
                          if ln.strip())
        h.update(code.encode())
    return h.hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled), or None when the summary is missing or
    was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("traffic-json:"):
                    rec = json.loads(line[len("traffic-json:"):])
                    break
            else:
                return None
    except OSError:
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else int(k["fetch_bytes"] + k["write_bytes"])


def _timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def _kernel_times(gal, fn, steps, torch):
    """Average duration per kernel from the dispatch timestamps (HIP events on
    the launch stream, recorded by the library)."""
    gal.timing.reset()
    gal.timing.enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    times = gal.timing.read()
    gal.timing.enable(False)
    gal.timing.reset()
    return {k: {"avg_us": 1e3 * ms / n, "launches": n} for k, (ms, n) in times.items()}


def stage_probe(gal, torch, dev, blocks=977, reps=50):
    """What a persistent kernel would pay per stage handoff: the same kernel
    (every block writes 8 KB, then one agent-scope atomic per block) without
    an atomic, with a relaxed, a release and an acquire-release one; average
    duration per launch (HIP events).  The release is the handoff a block
    needs to publish its stage output to the others."""
    ws = torch.zeros(gal.probe_stage_bytes(blocks), dtype=torch.uint8, device=dev)
    avg = {}
    for mode, name in enumerate(("none", "relaxed", "release", "acq_rel")):
        for _ in range(5):
            gal.probe_stage(mode, blocks, ws)
        t = _kernel_times(gal, lambda: gal.probe_stage(mode, blocks, ws), reps, torch)
        avg[name] = round(t[f"k_stage_probe<{mode}>"]["avg_us"], 3)
    return {"blocks": blocks, "threads_per_block": 256, "bytes_per_block": 8192, "avg_us": avg,
            "release_minus_relaxed_us": round(avg["release"] - avg["relaxed"], 3),
            "form": "k_stage_probe: every block writes its 8 KB slice, then one agent-scope "
                    "atomic add per block on a counter nothing waits on"}


def image_bench(gal, torch, np, dev, case, dtype, steps, warmup, grad=False, raw=False):
    """Plain chi2Image calls (one evaluation per call) on a case: evals/s,
    p50/p99 latency, per-kernel times and the dominant kernel's roofline; on
    a device-resident dataset, or with raw arrays (raw=True: the full
    spectrum, uv range checked per point).  grad: chi2Image + gradient."""
    p = 8 if dtype == torch.float64 else 4
    arr = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)
    img = arr(case.image)
    u, v = arr(case.u), arr(case.v)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=case.inc)
    model = gal.sampleImage(img, case.dxy, u, v, **kw)
    re = (model.real + arr(case.noise_re)).contiguous()
    im = (model.imag + arr(case.noise_im)).contiguous()
    w = arr(case.w)
    out = torch.empty((), dtype=torch.float64, device=dev)
    ds = None
    if raw:
        Q, P = case.N // 2 + 1, case.N // 2
        call = lambda: gal.chi2Image(img, case.dxy, u, v, re, im, w, out=out, **kw)
    else:
        ds = gal.Dataset(u, v, re, im, w)
        Q, P = ds.geometry(case.N, case.dxy)
        if grad:
            call = lambda: ds.chi2Image_grad(img, case.dxy, **kw)
        else:
            call = lambda: ds.chi2Image(img, case.dxy, out=out, **kw)
    ms = _timed(call, steps, warmup, torch)
    kern = _kernel_times(gal, call, max(steps // 4, 10), torch)
    lat = []
    for _ in range(min(steps, 200)):
        a = time.perf_counter()
        call()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    ab, fl = image_alg(case.N, case.M, Q, P, p)
    roof = kernel_roofline(kern, ab, fl)
    if ds is not None:
        ds.close()
    rnd = {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in x.items()}
           for k, x in kern.items()}
    return {"value": round(1e3 / ms, 1),
            "unit": "chi2+grad evals/s" if grad else "chi2 evals/s",
            "ms_per_eval": round(ms, 5),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                           "p99": round(float(np.percentile(lat, 99)), 4)},
            "dtype": "f64" if p == 8 else "f32", "Nxy": case.N, "M": case.M,
            "spectrum_cols_Q": Q, "spectrum_rows_P": P,
            "form": "raw arrays (full spectrum)" if raw else "device-resident dataset",
            "kernels": rnd, "roofline": roof}


def cube_bench(gal, torch, np, dev, steps, warmup):
    """The batched configuration: a 64-channel FP32 cube at 1024^2 (ragged M
    2e5..1e6, frequency-scaled uv sets) plus 32 FP32 chi2Image models of
    512^2..4096^2 (20 blobs each, each on its own observation, M 1e5..2e6), as
    one planned batch replayed from a HIP graph, against the same 96
    evaluations made one call at a time."""
    import workloads as wl

    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
    jobs, calls = [], []
    sizes = {}
    for c in list(wl.spectral_cube(64, 1024)) + list(wl.mixed_models(32)):
        ds = gal.Dataset(f32(c.u), f32(c.v), f32(c.noise_re), f32(c.noise_im), f32(c.w))
        img = f32(c.image)
        geo = torch.tensor([0.0, 1.0, c.inc, c.PA, c.dRA, c.dDec], dtype=torch.float64, device=dev)
        jobs.append({"ds": ds, "kind": gal.JOB_IMAGE, "Nxy": c.N, "dxy": c.dxy, "model": img,
                     "geo": geo})
        calls.append(lambda ds=ds, img=img, c=c: ds.chi2Image(img, c.dxy, c.PA, c.dRA, c.dDec,
                                                              c.inc))
        sizes[c.N] = sizes.get(c.N, 0) + 1
    b = gal.Batch(jobs)
    tuned = {N: gal.autotune_batch(b, N, torch.float32) for N in sorted(sizes)}
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        b.chi2()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.chi2()
    ms_graph = _timed(graph.replay, steps, warmup, torch)
    eager = b.chi2().clone()
    graph.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(eager, b.out))
    kern = _kernel_times(gal, b.chi2, max(steps // 4, 10), torch)
    ms_plain = _timed(lambda: [f() for f in calls], max(steps // 4, 10), 2, torch)
    n = len(jobs)
    info = b.info()
    M_tot = sum(j["ds"].M for j in jobs)
    b.close()
    for j in jobs:
        j["ds"].close()
    rnd = {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in x.items()}
           for k, x in kern.items()}
    return {"jobs": n, "fft_groups": info["fft_groups"], "sample_groups": info["sample_groups"],
            "batched": {"value": round(n * 1e3 / ms_graph, 1), "unit": "chi2 evals/s",
                        "ms_per_batch": round(ms_graph, 4), "form": "one HIP-graph replay",
                        "kernels": rnd},
            "plain": {"value": round(n * 1e3 / ms_plain, 1), "unit": "chi2 evals/s",
                      "ms_per_96_calls": round(ms_plain, 4)},
            "batched_vs_plain": round(ms_plain / ms_graph, 3), "fft_variants": tuned,
            "graph_replay_matches_eager": same, "models_per_size": sizes, "uv_points": M_tot,
            "workload": "64 channels at 1024^2 FP32 (frequency-scaled uv, M 2e5..1e6) + 32 FP32 "
                        "chi2Image models of 20 blobs at 512^2..4096^2, each on its own "
                        "observation (M 1e5..2e6)"}


def _serve_rate(Server, Request, ex, params, rate, n_req, warm, grad_frac, rng):
    """Poisson arrivals at `rate` of warm + n_req requests; statistics of the
    last n_req (the warm-up requests complete before the counters start)."""
    srv = Server(ex, max_batch=ex.max_batch, max_inflight=4).start()
    gaps = rng.exponential(1.0 / rate, n_req + warm)
    t_next = time.perf_counter()
    futs = []
    for i, prm in enumerate(params):
        t_next += gaps[i]
        while True:   # pace by sleeping: a spinning client would hold the GIL
            dt = t_next - time.perf_counter()
            if dt <= 0:
                break
            time.sleep(dt if dt > 2e-4 else 0)
        futs.append(srv.submit(Request(grad=bool(rng.random() < grad_frac), **prm)))
        if i == warm - 1:
            for f in futs:
                f.result(timeout=120)
            srv.reset_stats()
    for f in futs:
        f.result(timeout=300)
    srv.stop()
    st = srv.stats()
    return {"offered_req_per_s": rate,
            "evals_per_s": round(st["evals_per_s"], 1) if st["evals_per_s"] else None,
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "requests": st["completed"], "micro_batches": st["batches"],
            "host_launch_ms_per_batch": round(st["host_launch_ms_per_batch"], 3),
            "peak_hbm_MB": round(st["peak_hbm_bytes"] / 1e6, 1)}


def serve_bench(gal, torch, np, dev, rates, sat_rates, n_req, warm, grad_frac, n_datasets, max_M,
                max_batch=64):
    """Poisson stream of chi2Profile (+ gradient) requests against resident
    datasets, served by the continuous-batching loop; latency and throughput
    per arrival rate, then offered rates raised until the served rate falls
    behind (the loop's capacity)."""
    import workloads as wl
    from paper_1709_06999_amd.serve import GpuExecutor, Request, Server

    ex = GpuExecutor(dev, torch.float64, max_batch=max_batch, max_inflight=4)
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    # each dataset observes a fixed "true" profile at 2048^2 (model from the library) plus noise
    truth = wl.serve_requests(1, seed=1549)[0]
    Nm = 2048
    for dset in wl.serve_datasets(n_datasets, (100_000, max_M)):
        u, v = f64(dset["u"]), f64(dset["v"])
        Vm = gal.sampleProfile(f64(truth["I"]), truth["Rmin"], truth["dR"] * (truth["Nxy"] / Nm),
                               Nm, truth["dxy"], u, v, truth["inc"], truth["PA"])
        ex.add_dataset(dset["name"], dset["u"], dset["v"],
                       Vm.real.cpu().numpy() + dset["noise_re"],
                       Vm.imag.cpu().numpy() + dset["noise_im"], dset["w"])
    rng = np.random.default_rng(1550)
    out = {}
    for rate in rates:
        params = wl.serve_requests(n_req + warm, seed=int(1551 + rate))
        out[str(rate)] = _serve_rate(Server, Request, ex, params, rate, n_req, warm, grad_frac, rng)
    sat = {}
    for rate in sat_rates:
        params = wl.serve_requests(n_req + warm, seed=int(1551 + rate))
        r = _serve_rate(Server, Request, ex, params, rate, n_req, warm, grad_frac, rng)
        sat[str(rate)] = r
        if r["evals_per_s"] is None or r["evals_per_s"] < 0.95 * rate:
            break
    allr = list(out.values()) + list(sat.values())
    best = max(allr, key=lambda r: r["evals_per_s"] or 0.0)
    for d in ex.datasets.values():
        d.close()
    return {"workload": f"{n_datasets} resident datasets (M log-uniform in [1e5, {max_M:.0e}]), "
                        "requests: chi2Profile with Nxy in {512, 1024, 2048}, Nr in [512, 4096], "
                        f"{int(100 * grad_frac)}% with the adjoint gradient, Poisson arrivals",
            "per_rate": out, "saturation": sat,
            "capacity": {"evals_per_s": best["evals_per_s"], "at_offered": best["offered_req_per_s"],
                         "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"]}}


def served_headline(gal, torch, np, dev, case, n_req, warm, max_batch=64):
    """The served form at the headline workload: chi^2 requests of perturbed
    profiles (walkers) on the 2048^2, M = 1e6 dataset, all submitted at once
    (a closed batch, as an ensemble sampler's step), so that the loop runs at
    its capacity; evals/s and p50/p99 latency, to set beside the plain and
    batched forms of the same evaluation."""
    from paper_1709_06999_amd.serve import GpuExecutor, Request, Server

    ex = GpuExecutor(dev, torch.float64, max_batch=max_batch, max_inflight=4)
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    u, v = f64(case.u), f64(case.v)
    Vm = gal.sampleProfile(f64(case.I), case.Rmin, case.dR, case.N, case.dxy, u, v, case.inc,
                           case.PA, case.dRA, case.dDec)
    ex.add_dataset("p2048", case.u, case.v, Vm.real.cpu().numpy() + case.noise_re,
                   Vm.imag.cpu().numpy() + case.noise_im, case.w)
    rng = np.random.default_rng(1104)
    Ib = [case.I * (1.0 + 0.05 * rng.standard_normal(case.I.size)) for _ in range(64)]
    mk = lambda k: Request("p2048", Ib[k % 64], case.Rmin, case.dR, case.N, case.dxy,
                           inc=case.inc, PA=case.PA, dRA=case.dRA, dDec=case.dDec)
    srv = Server(ex, max_batch=max_batch, max_inflight=4).start()
    for f in [srv.submit(mk(k)) for k in range(warm)]:
        f.result(timeout=120)
    srv.reset_stats()
    futs = [srv.submit(mk(k)) for k in range(n_req)]
    for f in futs:
        f.result(timeout=300)
    srv.stop()
    st = srv.stats()
    ex.datasets["p2048"].close()
    return {"value": round(st["evals_per_s"], 1), "unit": "chi2 evals/s",
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "requests": st["completed"], "micro_batches": st["batches"],
            "host_launch_ms_per_batch": round(st["host_launch_ms_per_batch"], 3),
            "form": f"{n_req} chi2Profile requests (perturbed profiles) submitted at once to the "
                    f"continuous-batching loop (micro-batches of up to {max_batch}, 4 in flight), "
                    "2048^2, Nr=4096, M=1e6, FP64"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400, help="timed batched steps")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=64,
                    help="models (walkers) per batched step; 16 is also measured")
    ap.add_argument("--plain-steps", type=int, default=2000)
    ap.add_argument("--latency-samples", type=int, default=300)
    ap.add_argument("--grad-steps", type=int, default=300, help="timed plain gradient calls")
    ap.add_argument("--no-cube", action="store_true",
                    help="skip the batched cube + mixed-models section")
    ap.add_argument("--field-sources", type=int, default=16,
                    help="sources in the field section (copies of the profile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch batches without a HIP graph")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (a known-size kernel for "
                         "scaling HBM byte counters)")
    ap.add_argument("--fft-variants", default=None,
                    help="fixed FFT variants rows_image,cols,rows_sym,cols_sym (0: E=16, 1: E=8, "
                         "2: E=4) instead of autotuning, e.g. for counter runs that must see "
                         "the same kernels")
    ap.add_argument("--fft-variants-batch", default=None,
                    help="fixed FFT variants for the batched sections (default: as "
                         "--fft-variants, else autotuned on the batch)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-load section")
    ap.add_argument("--stage-probe", action="store_true",
                    help="run only the stage-handoff probe (what a persistent kernel pays per "
                         "stage) and print its JSON")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the served-load section and print its JSON (profiling aid)")
    ap.add_argument("--serve-rates", default="100,200,500,1000,2000,5000",
                    help="Poisson arrival rates (requests/s) of the served-load section")
    ap.add_argument("--serve-requests", type=int, default=2000, help="timed requests per rate")
    ap.add_argument("--serve-max-batch", type=int, default=64,
                    help="largest micro-batch of the served-load section")
    ap.add_argument("--saturation-rates", default="10000,20000,50000,100000",
                    help="offered rates above the sweep, raised until the served rate falls "
                         "behind the offered one")
    ap.add_argument("--no-images", action="store_true",
                    help="skip the chi2Image sections (256^2, 2048^2 with gradient, 4096^2 "
                         "FP64 / FP32)")
    ap.add_argument("--kind", choices=["profile", "image"], default="profile",
                    help="plain path: chi2Profile (default) or chi2Image of the swept image")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              "single-device by design.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    _ensure_built()
    import paper_1709_06999_amd as gal
    import workloads as wl

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    gal.init(0)
    rates = [int(r) for r in args.serve_rates.split(",")]
    sat_rates = [int(r) for r in args.saturation_rates.split(",")] if args.saturation_rates else []
    if args.stage_probe:
        print(json.dumps({"stage_probe": stage_probe(gal, torch, dev)}), flush=True)
        return
    if args.serve_only:
        served = serve_bench(gal, torch, np, dev, rates, sat_rates, args.serve_requests, 200, 0.5,
                             8, 2_000_000, args.serve_max_batch)
        print(json.dumps({"served": served}), flush=True)
        return
    case = wl.profile_2048()
    N, M, Nr = case.N, case.M, case.I.size
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    I, u, v = f64(case.I), f64(case.u), f64(case.v)
    geo = dict(inc=case.inc, PA=case.PA, dRA=case.dRA, dDec=case.dDec)
    # observed visibilities: the library's own model plus seeded noise
    model = gal.sampleProfile(I, case.Rmin, case.dR, N, case.dxy, u, v, **geo)
    re = (model.real + f64(case.noise_re)).contiguous()
    im = (model.imag + f64(case.noise_im)).contiguous()
    w = f64(case.w)
    ds = gal.Dataset(u, v, re, im, w)
    Q, P = ds.geometry(N, case.dxy)
    # FFT schedules for this image size and the reachable part of the spectrum
    frac = ds.rho_max * N * case.dxy / (N / 2 - 1)
    tune_times = {}
    if args.fft_variants:
        tuned = [int(x) for x in args.fft_variants.split(",")]
        gal.tune_set(N, tuned, torch.float64)
    else:
        tuned = gal.autotune(N, torch.float64, frac, times=tune_times)

    if args.calib_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    progress("plain chi2Profile")
    # ---- plain: one evaluation per call --------------------------------
    out = torch.empty((), dtype=torch.float64, device=dev)
    if args.kind == "profile":
        plain = lambda: ds.chi2Profile(I, case.Rmin, case.dR, N, case.dxy, out=out, **geo)
    else:
        img = gal.sweep(I, case.Rmin, case.dR, N, case.dxy, case.inc)
        plain = lambda: ds.chi2Image(img, case.dxy, case.PA, case.dRA, case.dDec, out=out)
    ms_plain = _timed(plain, args.plain_steps, args.warmup, torch)
    chi2_val = float(out)
    kern_plain = _kernel_times(gal, plain, args.plain_steps, torch)
    lat = []
    for _ in range(args.latency_samples):
        a = time.perf_counter()
        plain()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.sort(np.array(lat))

    progress("plain gradient")
    # ---- plain gradient: chi^2 and d chi^2 / d I per call ------------------
    grad_call = lambda: ds.chi2Profile_grad(I, case.Rmin, case.dR, N, case.dxy, **geo)
    ms_grad = _timed(grad_call, args.grad_steps, args.warmup, torch)
    kern_grad = _kernel_times(gal, grad_call, max(args.grad_steps // 3, 20), torch)

    # ---- plain geometry gradient: chi^2 and d chi^2 / d (PA, dRA, dDec, inc) ----
    geo_call = lambda: ds.chi2Profile_geograd(I, case.Rmin, case.dR, N, case.dxy, **geo)
    ms_geo = _timed(geo_call, args.grad_steps, args.warmup, torch)

    progress("field of sources")
    # ---- a field of several sources (Sec. 3.2): copies of the profile at
    # other offsets and orientations, one scene; with the copies reading the
    # first one's spectrum, and with a transform per copy --------------------
    S = args.field_sources
    src_o = wl.field_of_copies(case, S, seed=1103)
    shared = []
    for s in src_o:
        d = {k: x for k, x in s.items() if k != "I"}
        d["model"] = I if s.get("share") is None else None
        shared.append(d)
    own = [dict(d, model=I, share=None, Rmin=case.Rmin, dR=case.dR, inc=case.inc) for d in shared]
    fb_shared, fb_own = gal.Batch(ds._scene_jobs(shared)), gal.Batch(ds._scene_jobs(own))
    ms_field = _timed(fb_shared.chi2, args.grad_steps, args.warmup, torch)
    kern_field = _kernel_times(gal, fb_shared.chi2, max(args.grad_steps // 3, 20), torch)
    ms_field_own = _timed(fb_own.chi2, args.grad_steps, args.warmup, torch)
    field_c2 = float(fb_shared.chi2()[0])
    field_match = abs(float(fb_own.chi2()[0]) - field_c2) <= 1e-12 * abs(field_c2)
    ms_field_call = _timed(lambda: ds.chi2Sources(shared), max(args.grad_steps // 3, 20),
                           args.warmup, torch)
    fb_shared.close()
    fb_own.close()

    progress("cube + mixed models")
    # ---- the batched configuration: cube + mixed models in one graph ------
    cube = None if args.no_cube else cube_bench(gal, torch, np, dev, max(args.steps // 4, 20),
                                                args.warmup)

    progress("batched walkers (headline)")
    # ---- batched: K walkers (different profiles and geometry) per step ----
    tuned_plain = list(tuned)

    def walkers(K):
        """A step of K walkers replayed from a HIP graph: (batch, models, ms per
        step, per-kernel times, replay matches eager, FFT variants, tuning times)."""
        rng = np.random.default_rng(1102)
        Ib = f64(np.stack([case.I * (1.0 + 0.05 * rng.standard_normal(Nr)) for _ in range(K)]))
        geob = f64(np.array([[case.Rmin, case.dR, case.inc + 0.05 * rng.standard_normal(),
                              case.PA + 0.05 * rng.standard_normal(),
                              0.1 * case.dxy * rng.standard_normal(),
                              0.1 * case.dxy * rng.standard_normal()] for _ in range(K)]))
        batch = gal.profile_batch(ds, Ib, geob, N, case.dxy)
        tune_ms = {}
        if args.fft_variants_batch:
            tv = [int(x) for x in args.fft_variants_batch.split(",")]
            gal.tune_set(N, tv, torch.float64)
        elif not args.fft_variants:
            tv = gal.autotune_batch(batch, N, torch.float64, times=tune_ms)
        else:
            tv = list(tuned)
        step = batch.chi2
        if not args.no_graph:
            side = torch.cuda.Stream(device=dev)
            side.wait_stream(torch.cuda.current_stream(dev))
            with torch.cuda.stream(side):
                batch.chi2()                      # warm-up outside the capture
            torch.cuda.current_stream(dev).wait_stream(side)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                batch.chi2()
            step = graph.replay
        ms = _timed(step, args.steps, args.warmup, torch)
        # every replay matches an eager execution
        replayed = batch.out.clone()
        eager = batch.chi2().clone()
        torch.cuda.synchronize()
        ok = bool(torch.equal(eager, replayed))
        kt = _kernel_times(gal, batch.chi2, max(args.steps // 4, 20), torch)
        return batch, Ib, ms, kt, ok, tv, tune_ms

    # 16 walkers (the form of earlier measurements), then the headline's K
    b16 = None
    if args.batch != 16:
        bt, _, ms16, kt16, ok16, tv16, _ = walkers(16)
        b16 = {"value": round(16 * 1e3 / ms16, 1), "unit": "chi2 evals/s",
               "ms_per_step": round(ms16, 5), "batch": 16, "fft_variants": tv16,
               "graph_replay_matches_eager": ok16,
               "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                               for kk, vv in x.items()} for k, x in kt16.items()}}
        bt.close()
    K = args.batch
    batch, Ib, ms_batch, kern, replay_ok, tuned, batch_tune_ms = walkers(K)
    chi2_batch = batch.out.cpu().numpy()
    evals_per_s = K * 1e3 / ms_batch

    progress("batched gradients")
    # ---- batched with gradients: the same K walkers, one batch_exec call ---
    gbuf = [torch.empty_like(Ib[k]) for k in range(K)]
    gjobs = batch.jobs
    gstep = lambda: gal.batch_exec(gjobs, gbuf)
    ms_bgrad = _timed(gstep, max(args.steps // 4, 20), args.warmup, torch)
    kern_bgrad = _kernel_times(gal, gstep, 20, torch)

    # ---- roofline of the dominant kernel of the batched step ---------------
    ab = algorithmic_bytes(N, Nr, M, Q, P, "profile")
    Qe = Q + (Q & 1)
    spec = (P + 1) * Qe * 8
    ab_batch = {"kb_rows_sym": K * ab["k_rows_sym"], "kb_rows_even": K * ab["k_rows_sym"],
                "kb_cols_sym": K * ab["k_cols_sym"], "kb_cols_even": K * ab["k_cols_sym"],
                "kb_sample_sym_chi2": 5 * 8 * M + K * spec, "kb_reduce": K * ab["k_reduce"]}
    for k in kern:
        if k in ab_batch:
            kern[k]["alg_bytes"] = ab_batch[k]
            kern[k]["alg_GBps"] = ab_batch[k] / (kern[k]["avg_us"] * 1e-6) / 1e9
    for k in kern_plain:
        if k in ab:
            kern_plain[k]["alg_bytes"] = ab[k]
            kern_plain[k]["alg_GBps"] = ab[k] / (kern_plain[k]["avg_us"] * 1e-6) / 1e9
    fl_batch = {**fft_flops(N, Q, K), **sample_flops(M, K)}
    for k in kern:
        if k in fl_batch:
            kern[k]["alg_flops"] = fl_batch[k]
            kern[k]["alg_TFLOPs"] = fl_batch[k] / (kern[k]["avg_us"] * 1e-6) / 1e12
    fl_plain = {**fft_flops(N, Q, 1), **sample_flops(M, 1)}
    for k in kern_plain:
        kk = k.replace("k_", "kb_", 1)
        if kk in fl_plain:
            kern_plain[k]["alg_flops"] = fl_plain[kk]
            kern_plain[k]["alg_TFLOPs"] = fl_plain[kk] / (kern_plain[k]["avg_us"] * 1e-6) / 1e12
    dom = max((k for k in kern if k in ab_batch), key=lambda k: kern[k]["avg_us"])
    if dom in fl_batch:
        # FFT passes, and the sampler with K jobs per point: FP64 arithmetic and
        # its issue bound them (their HBM bytes take far less)
        achieved = kern[dom]["alg_TFLOPs"]
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                    "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                    "traffic": stored_traffic(dom), "alg_flops_per_launch": fl_batch[dom],
                    "alg_bytes_per_launch": ab_batch[dom],
                    "hbm_frac": round(kern[dom]["alg_GBps"] / HBM_PEAK_GBS, 4)}
    else:
        achieved = kern[dom]["alg_GBps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": stored_traffic(dom), "alg_bytes_per_launch": ab_batch[dom]}
    step_bytes = sum(ab_batch[k] for k in kern if k in ab_batch)  # the kernels the step ran
    roofline["step_alg_bytes"] = step_bytes
    roofline["step_hbm_frac"] = round(step_bytes / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    pb = path_bytes(N, Nr, M)
    unpruned = {
        "definition": "evals/s x the bytes of one evaluation counted without pruning, the "
                      "even form or batching (full half spectrum written and read twice, "
                      "every observation read per evaluation), over 8 TB/s.  Not a roofline "
                      "fraction: the kernels do not move these bytes (see roofline)",
        "bytes_per_eval": pb,
        "plain": round(1e3 / ms_plain * pb["chi2"] / 1e9 / HBM_PEAK_GBS, 4),
        "batched": round(evals_per_s * pb["chi2"] / 1e9 / HBM_PEAK_GBS, 4),
        "plain_grad": round(1e3 / ms_grad * pb["chi2_grad"] / 1e9 / HBM_PEAK_GBS, 4),
        "batched_grad": round(K * 1e3 / ms_bgrad * pb["chi2_grad"] / 1e9 / HBM_PEAK_GBS, 4),
    }

    progress("served load")
    served = None
    if not args.no_serve:
        served = serve_bench(gal, torch, np, dev, rates, sat_rates, args.serve_requests, 200, 0.5,
                             8, 2_000_000, args.serve_max_batch)
        for key, mb in (("headline", 64), ("headline_mb16", 16)):
            served[key] = served_headline(gal, torch, np, dev, case, 8000, 500, mb)
            served[key]["served_vs_plain"] = round(served[key]["value"] / (1e3 / ms_plain), 3)

    progress("chi2Image sections")
    images = None
    if not args.no_images:
        isteps = max(args.grad_steps // 2, 50)
        images = {
            "gaussian_256_M1e4": image_bench(gal, torch, np, dev, wl.gaussian_image_256(),
                                             torch.float64, isteps, args.warmup),
            "blobs_2048_M1e6": image_bench(gal, torch, np, dev, wl.image_2048(), torch.float64,
                                           isteps, args.warmup),
            "blobs_2048_M1e6_grad": image_bench(gal, torch, np, dev, wl.image_2048(),
                                                torch.float64, isteps // 2, args.warmup,
                                                grad=True),
        }
        b4 = wl.blobs_4096()
        images["blobs_4096_M5e6_f64"] = image_bench(gal, torch, np, dev, b4, torch.float64,
                                                    isteps // 2, args.warmup)
        images["blobs_4096_M5e6_f32"] = image_bench(gal, torch, np, dev, b4, torch.float32,
                                                    isteps // 2, args.warmup)
        del b4

    progress("oracle baseline")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        nre, nim = case.noise_re, case.noise_im   # values do not change the oracle's cost
        t_runs = []
        start = time.perf_counter()
        while len(t_runs) < 3 and (time.perf_counter() - start) < 20.0:
            a = time.perf_counter()
            oracle.chi2Profile(case.I, case.Rmin, case.dR, N, case.dxy, case.u, case.v, nre, nim,
                               case.w, case.inc, case.PA, case.dRA, case.dDec)
            t_runs.append(time.perf_counter() - a)
        cores = oracle.num_threads()
        cpu = {"value": round(1.0 / float(np.median(t_runs)), 5), "unit": "chi2 evals/s",
               "cores": cores, "kind": "oracle",
               "sample": f"{len(t_runs)} full evaluation(s) of this workload by the FP64 "
                         "direct-DFT oracle (O(N^3)), median time",
               "nproc": os.cpu_count(),
               "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
        # one thread: the 256^2 chi2Image workload (median of 3) and this one (one run)
        c0 = wl.gaussian_image_256()
        oracle.set_num_threads(1)
        try:
            t0 = []
            for _ in range(3):
                a = time.perf_counter()
                oracle.chi2Image(c0.image, c0.dxy, c0.u, c0.v, c0.noise_re, c0.noise_im, c0.w,
                                 c0.PA, c0.dRA, c0.dDec, c0.inc)
                t0.append(time.perf_counter() - a)
            a = time.perf_counter()
            oracle.chi2Profile(case.I, case.Rmin, case.dR, N, case.dxy, case.u, case.v, nre, nim,
                               case.w, case.inc, case.PA, case.dRA, case.dDec)
            t1 = time.perf_counter() - a
        finally:
            oracle.set_num_threads(cores)
        cpu["one_thread"] = {"chi2Image_256_M1e4_evals_per_s": round(1.0 / float(np.median(t0)), 4),
                             "chi2Profile_2048_M1e6_evals_per_s": round(1.0 / t1, 5)}

    rnd = lambda d: {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                         for kk, vv in x.items()} for k, x in d.items()}
    res = {
        "metric": METRIC,
        "value": round(evals_per_s, 1),
        "unit": "chi2 evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batch, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"chi2Profile 2048^2, Nr=4096, M=1e6 uv, FP64; a step is one "
                               f"batch of {K} models (walkers) on a device-resident dataset"
                               + ("" if args.no_graph else ", replayed from a HIP graph"),
                   "Nxy": N, "Nr": int(Nr), "M": M, "batch": K, "spectrum_cols_Q": Q,
                   "spectrum_rows_P": P, "fft_variants": tuned,
                   "fft_variants_plain": tuned_plain, "fft_variant_ms": tune_times,
                   "fft_variant_batch_ms": batch_tune_ms,
                   "graph_replay_matches_eager": replay_ok,
                   "chi2_first_walker": float(chi2_batch[0])},
        "plain": {"value": round(1e3 / ms_plain, 1), "unit": "chi2 evals/s",
                  "ms_per_eval": round(ms_plain, 5), "kind": args.kind, "chi2": chi2_val,
                  "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                                 "p99": round(float(np.percentile(lat, 99)), 4)},
                  "kernels": rnd(kern_plain)},
        "batched_vs_plain": round(evals_per_s / (1e3 / ms_plain), 3),
        "batch_16": b16,
        "grad": {"plain": {"value": round(1e3 / ms_grad, 1), "unit": "chi2+grad evals/s",
                           "ms_per_eval": round(ms_grad, 5), "kernels": rnd(kern_grad)},
                 "batched": {"value": round(K * 1e3 / ms_bgrad, 1), "unit": "chi2+grad evals/s",
                             "ms_per_step": round(ms_bgrad, 5), "batch": K,
                             "form": "one gal_batch_exec call per step (planned at the call)",
                             "kernels": rnd(kern_bgrad)},
                 "geometry_plain": {"value": round(1e3 / ms_geo, 1),
                                    "unit": "chi2 + d/d(PA, dRA, dDec, inc) evals/s",
                                    "ms_per_eval": round(ms_geo, 5)}},
        "cube": cube,
        "field": {"sources": S,
                  "shared_spectrum": {"value": round(1e3 / ms_field, 1), "unit": "field chi2 evals/s",
                                      "ms_per_eval": round(ms_field, 5),
                                      "kernels": rnd(kern_field)},
                  "transform_per_source": {"value": round(1e3 / ms_field_own, 1),
                                           "unit": "field chi2 evals/s",
                                           "ms_per_eval": round(ms_field_own, 5)},
                  "sharing_gain": round(ms_field_own / ms_field, 3),
                  "one_shot_call_ms": round(ms_field_call, 5),
                  "same_chi2": field_match,
                  "form": f"{S} copies of the 2048^2 profile (one scene) on the M=1e6 dataset; "
                          "persistent plan, one gal_batch_chi2 per evaluation"},
        "evals_vs_unpruned_bytes": unpruned,
        "stage_probe": stage_probe(gal, torch, dev),
        "served": served,
        "images": images,
        "kernels": rnd(kern),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": {"gtx1060_chi2Profile_2048_ms": 18.0,
                          "note": "paper GPU time includes per-call host-to-device copies"},
    }
    batch.close()
    ds.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
