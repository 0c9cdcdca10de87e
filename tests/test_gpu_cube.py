"""The batched configuration at full size: a spectral cube of 64 channels at
1024^2 FP32 (each channel its own uv set, scaled by frequency, ragged M from
2e5 to 1e6) plus 32 chi2Image models of mixed sizes (512^2 to 4096^2, 20
Gaussian blobs each, each on its own observation of M in 1e5..2e6) in one
planned batch, replayed from a HIP graph.  Every job against its single call,
every replay against an eager execution (with eager work in between), two
channels and one mixed model of every size against the oracle."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import assert_vis_close, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu

F = np.float32


def _obs_dataset(gal, dev, u, v, V, nre, nim, w):
    re, im = rounded(V.real + nre, F), rounded(V.imag + nim, F)
    ds = gal.Dataset(*(t(a, F, dev) for a in (u, v, re, im, w)))
    return ds, re, im


def _image_job(gal, dev, torch, c, oracle_model, full_oracle):
    """A dataset whose observations are 1.02 x a model + noise (so chi^2 is
    not at the noise floor): the oracle's model for checked jobs
    (full_oracle: every point, else None), the library's own single-call
    visibilities for the others."""
    img = t(c.image, F, dev)
    u32, v32 = rounded(c.u, F), rounded(c.v, F)
    check = None
    if oracle_model and full_oracle:
        Vo = oracle.sampleImage(rounded(c.image, F), c.dxy, u32, v32, c.PA, c.dRA, c.dDec, 0.0)
        ds, re, im = _obs_dataset(gal, dev, u32, v32, 1.02 * Vo, c.noise_re, c.noise_im, c.w)
        check = (Vo, re, im)
    else:
        ds0 = gal.Dataset(t(u32, F, dev), t(v32, F, dev))
        Vg = ds0.sampleImage(img, c.dxy, c.PA, c.dRA, c.dDec).cpu().numpy().astype(np.complex128)
        ds0.close()
        ds, _, _ = _obs_dataset(gal, dev, u32, v32, 1.02 * Vg, c.noise_re, c.noise_im, c.w)
        if oracle_model:
            check = "sampled"
    geo = torch.tensor([0.0, 1.0, c.inc, c.PA, c.dRA, c.dDec], dtype=torch.float64, device=dev)
    job = {"ds": ds, "kind": gal.JOB_IMAGE, "Nxy": c.N, "dxy": c.dxy, "model": img, "geo": geo}
    return job, check


def test_cube_and_mixed_models_in_one_graph_launch():
    dev = device()
    import torch

    import paper_1709_06999_amd as gal

    jobs, cases, checks = [], [], {}
    for k, c in enumerate(wl.spectral_cube(64, 1024)):
        job, chk = _image_job(gal, dev, torch, c, k in (0, 63), True)
        if chk is not None:
            checks[len(jobs)] = chk
        jobs.append(job)
        cases.append(c)
    first_mixed = len(jobs)
    seen = set()
    for c in wl.mixed_models(32):
        first_of_size = c.N not in seen
        seen.add(c.N)
        print(f"mixed model {len(jobs) - first_mixed}: N={c.N} M={c.M}", flush=True)
        job, chk = _image_job(gal, dev, torch, c, first_of_size, c.N <= 2048)
        if chk is not None:
            checks[len(jobs)] = chk
        jobs.append(job)
        cases.append(c)
    assert seen == {512, 1024, 2048, 4096}
    b = gal.Batch(jobs)
    info = b.info()
    assert info["jobs"] == 96 and info["sample_groups"] == 96
    gal.autotune_batch(b, 1024, torch.float32)
    eager = b.chi2().clone()
    # graph capture on a side stream, then replays with eager work between
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        b.chi2()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.chi2()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.out, eager), rep
        b.chi2(out=torch.empty_like(eager))  # eager work between replays
        torch.cuda.synchronize()
    c2 = eager.cpu().numpy()
    # every job against its single call
    for i, j in enumerate(jobs):
        g = j["geo"].cpu().numpy()
        c2s = float(j["ds"].chi2Image(j["model"], j["dxy"], g[3], g[4], g[5], g[2]))
        assert abs(c2[i] - c2s) <= 1e-6 * c2s, (i, c2[i], c2s)
    # checked jobs against the oracle: every visibility and chi^2 within the
    # bound of the measured model error plus its FP32 rounding; the 4096^2
    # model at sampled points (the oracle's per-node double sums)
    for i, chk in checks.items():
        c = cases[i]
        Vg = jobs[i]["ds"].sampleImage(jobs[i]["model"], c.dxy, c.PA, c.dRA,
                                       c.dDec).cpu().numpy()
        if chk == "sampled":
            rho = np.hypot(c.u, c.v)
            order = np.argsort(rho)
            pick = np.unique(np.concatenate([order[:4], order[-4:], np.random.default_rng(
                1499).choice(c.M, 8, replace=False)]))
            Vo = oracle.sample_direct(rounded(c.image, F), c.dxy, rounded(c.u[pick], F),
                                      rounded(c.v[pick], F), c.PA, c.dRA, c.dDec, 0.0)
            flux = abs(float(np.sum(rounded(c.image, F))))
            err = np.max(np.abs(Vg[pick] - Vo))
            print(f"job {i} (N={c.N}): sampled max|dV| {err:.3e}, flux {flux:.3e}", flush=True)
            assert err <= 1e-4 * max(np.max(np.abs(Vo)), flux)
            continue
        Vo, re, im = chk
        err = assert_vis_close(Vg, Vo, F, f"batched job {i} (N={c.N})")
        c2o = oracle.chi2(Vo, re, im, rounded(c.w, F))
        dV = np.abs(Vg - Vo) + np.abs(Vg) * 2.0 ** -23
        print(f"job {i} (N={c.N}, M={c.M}): max|dV|/max|V| {err:.3e}; chi2 {c2[i]:.9g} "
              f"oracle {c2o:.9g}", flush=True)
        assert abs(c2[i] - c2o) <= chi2_bound(c2o, dV, c.w), (i, c2[i], c2o)
    b.close()
    for j in jobs:
        j["ds"].close()
