"""The batched configuration at full size: a spectral cube of 64 channels at
1024^2 FP32 (each channel its own uv set, scaled by frequency, ragged M from
2e5 to 1e6) plus 32 models of mixed sizes (512^2 to 4096^2) in one planned
batch, replayed from a HIP graph.  Every job against its single call, every
replay against an eager execution (with eager work in between), and a few
jobs against the oracle."""
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


def test_cube_and_mixed_models_in_one_graph_launch():
    dev = device()
    import torch

    import paper_1709_06999_amd as gal

    jobs, keep, checks = [], [], {}
    # 64 channels: observed = a model shifted in flux (so chi^2 is not at the
    # noise floor) + noise; the GPU's own single-call visibilities stand in for
    # the model of most channels, the oracle's for the checked ones
    for k, c in enumerate(wl.spectral_cube(64, 1024)):
        img = t(c.image, F, dev)
        u32, v32 = rounded(c.u, F), rounded(c.v, F)
        if k in (0, 63):
            Vo = oracle.sampleImage(rounded(c.image, F), c.dxy, u32, v32, c.PA, c.dRA, c.dDec, 0.0)
            ds, re, im = _obs_dataset(gal, dev, u32, v32, 1.02 * Vo, c.noise_re, c.noise_im, c.w)
            checks[len(jobs)] = (Vo, re, im, c)
        else:
            ds0 = gal.Dataset(t(u32, F, dev), t(v32, F, dev))
            Vg = ds0.sampleImage(img, c.dxy, c.PA).cpu().numpy().astype(np.complex128)
            ds0.close()
            ds, _, _ = _obs_dataset(gal, dev, u32, v32, 1.02 * Vg, c.noise_re, c.noise_im, c.w)
        geo = torch.tensor([0.0, 1.0, c.inc, c.PA, c.dRA, c.dDec], dtype=torch.float64, device=dev)
        jobs.append({"ds": ds, "kind": gal.JOB_IMAGE, "Nxy": c.N, "dxy": c.dxy, "model": img,
                     "geo": geo})
        keep.append((ds, img, geo))
    # 32 mixed models on two shared datasets
    sets, models = wl.mixed_models(32)
    dsets = []
    for (u, v, nre, nim, w) in sets:
        ds, _, _ = _obs_dataset(gal, dev, rounded(u, F), rounded(v, F), np.zeros(u.size), nre, nim,
                                w)
        dsets.append(ds)
    first_mixed = len(jobs)
    for m in models:
        I = t(m["I"], F, dev)
        geo = torch.tensor([m["Rmin"], m["dR"], m["inc"], m["PA"], m["dRA"], m["dDec"]],
                           dtype=torch.float64, device=dev)
        jobs.append({"ds": dsets[m["set"]], "kind": gal.JOB_PROFILE, "Nxy": m["N"], "dxy": m["dxy"],
                     "model": I, "geo": geo})
        keep.append((I, geo))
    b = gal.Batch(jobs)
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
        if j["kind"] == gal.JOB_IMAGE:
            c2s = float(j["ds"].chi2Image(j["model"], j["dxy"], g[3], g[4], g[5], g[2]))
        else:
            c2s = float(j["ds"].chi2Profile(j["model"], g[0], g[1], j["Nxy"], j["dxy"], g[2], g[3],
                                            g[4], g[5]))
        assert abs(c2[i] - c2s) <= 1e-6 * c2s, (i, c2[i], c2s)
    # the two checked channels against the oracle (chi^2 within the bound of
    # the measured model error plus its FP32 rounding)
    for i, (Vo, re, im, c) in checks.items():
        Vg = jobs[i]["ds"].sampleImage(jobs[i]["model"], c.dxy, c.PA).cpu().numpy()
        assert_vis_close(Vg, Vo, F, f"cube channel {i}")
        c2o = oracle.chi2(Vo, re, im, rounded(c.w, F))
        dV = np.abs(Vg - Vo) + np.abs(Vg) * 2.0 ** -23
        assert abs(c2[i] - c2o) <= chi2_bound(c2o, dV, c.w), (i, c2[i], c2o)
    # the largest mixed model against the oracle's direct sums at sampled points
    big = max(range(len(models)), key=lambda i: models[i]["N"])
    m = models[big]
    u, v = sets[m["set"]][0], sets[m["set"]][1]
    pick = np.random.default_rng(1701).choice(u.size, 8, replace=False)
    img = oracle.sweep(rounded(m["I"], F), m["Rmin"], m["dR"], m["N"], m["dxy"], m["inc"])
    Vo = oracle.sample_direct(img, m["dxy"], rounded(u[pick], F), rounded(v[pick], F), m["PA"],
                              m["dRA"], m["dDec"], 0.0)
    flux = abs(float(np.sum(img)))
    del img
    Vg = dsets[m["set"]].sampleProfile(jobs[first_mixed + big]["model"], m["Rmin"], m["dR"], m["N"],
                                       m["dxy"], m["inc"], m["PA"], m["dRA"],
                                       m["dDec"]).cpu().numpy()
    assert np.max(np.abs(Vg[pick] - Vo)) <= 1e-4 * flux
    b.close()
