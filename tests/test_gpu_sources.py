"""Fields of several sources (scenes): visibilities, chi^2 and gradients of the
summed model against the oracle; scenes mixed with single jobs in one call,
each result the same as alone; sharing a spectrum; datasets without
observations; the plan's checks."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import assert_vis_close, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu


def _gal():
    import paper_1709_06999_amd as gal

    return gal


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _field(seed, dtype, N_img=128, N_prof=256, M=20000):
    """A field on one uv set: an image source (N_img), a profile (N_prof), two
    copies of the profile elsewhere (sharing its spectrum) and a second,
    smaller image with its own grid.  Returns (oracle sources, gpu sources,
    uv, noise, weights) with the models rounded to ``dtype``."""
    p = wl.random_case(N_prof, M, seed=seed, kind="profile", fill=0.5)
    a = wl.random_case(N_img, 10, seed=seed + 1)
    b = wl.random_case(N_img // 2, 10, seed=seed + 2)
    rng = np.random.default_rng(seed + 3)
    # every source's grid reaches the uv radius: pixel sizes set from the profile's
    dxy_a = p.dxy * N_prof / N_img * 0.9
    dxy_b = p.dxy * N_prof / (N_img // 2) * 0.45
    img_a, img_b = rounded(a.image, dtype), rounded(b.image, dtype)
    # the profile's pixels about as bright as the image's (pixel value = I dxy^2)
    I = rounded(p.I / np.max(p.I) * np.max(np.abs(a.image)) / p.dxy ** 2, dtype)
    geo = lambda: dict(PA=rng.uniform(0, np.pi), dRA=rng.normal(0, 4 * p.dxy),
                       dDec=rng.normal(0, 4 * p.dxy))
    o = [dict(kind="image", image=img_a, dxy=dxy_a, inc=0.3, **geo()),
         dict(kind="profile", I=I, Rmin=p.Rmin, dR=p.dR, Nxy=N_prof, dxy=p.dxy, inc=0.6, **geo()),
         dict(kind="profile", I=None, inc=0.0, share=1, **geo()),
         dict(kind="profile", I=None, inc=0.0, share=1, **geo()),
         dict(kind="image", image=img_b, dxy=dxy_b, inc=0.1, **geo())]
    g = []
    for s in o:
        d = {k: v for k, v in s.items() if k not in ("image", "I")}
        if s["kind"] == "image":
            d["model"] = s["image"]
        else:
            d["model"] = s["I"]
            d.setdefault("Nxy", N_prof)
            d.setdefault("dxy", p.dxy)
        g.append(d)
    u, v = rounded(p.u, dtype), rounded(p.v, dtype)
    return o, g, u, v, p.noise_re, p.noise_im, rounded(p.w, dtype)


def _gpu_sources(g, dtype, dev):
    out = []
    for s in g:
        d = dict(s)
        d["model"] = None if s["model"] is None else t(s["model"], dtype, dev)
        out.append(d)
    return out


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_field_matches_oracle(dtype):
    dev = device()
    gal = _gal()
    o, g, u, v, nre, nim, w = _field(5100, dtype)
    Vo = oracle.sample_sources(o, u, v)
    # observations off the model by 30%: residuals well above FP32 rounding
    re, im = rounded(1.3 * Vo.real + nre, dtype), rounded(0.7 * Vo.imag + nim, dtype)
    ds = gal.Dataset(*(t(a, dtype, dev) for a in (u, v, re, im, w)))
    src = _gpu_sources(g, dtype, dev)
    Vg = ds.sampleSources(src).cpu().numpy()
    assert_vis_close(Vg, Vo, dtype, "field")
    c2o, go = oracle.grad_sources(o, u, v, re, im, w)
    c2g, gg = ds.chi2Sources(src, grad=True)
    assert abs(float(c2g) - c2o) <= chi2_bound(c2o, Vg - Vo, w) + (1e-6 * c2o if dtype == np.float32 else 0)
    tol = 1e-8 if dtype == np.float64 else 1e-3
    for k, (a, b) in enumerate(zip(gg, go)):
        if b is None:
            assert a is None
            continue
        assert _rel(a.cpu().numpy().astype(np.float64), b) <= tol, k
    # the chi^2-only call gives the same chi^2 (its points are summed in
    # another order: strided instead of consecutive per thread)
    c2_only = float(ds.chi2Sources(src))
    assert abs(c2_only - float(c2g)) <= 1e-12 * abs(float(c2g))


def test_field_in_a_mixed_call_equals_alone():
    # scenes (with and without gradients) and single jobs in one call, on two
    # datasets: every entry equals its own call
    dev = device()
    gal = _gal()
    import torch

    d = np.float64
    o, g, u, v, nre, nim, w = _field(5200, d)
    Vo = oracle.sample_sources(o, u, v)
    re, im = Vo.real + nre, Vo.imag + nim
    ds = gal.Dataset(*(t(a, d, dev) for a in (u, v, re, im, w)))
    c2_alone, g_alone = ds.chi2Sources(_gpu_sources(g, d, dev), grad=True)
    single = wl.random_case(256, 9000, seed=5201, kind="profile", fill=0.8)
    Vs = oracle.sampleProfile(single.I, single.Rmin, single.dR, single.N, single.dxy, single.u,
                              single.v, single.inc, single.PA, single.dRA, single.dDec)
    ds2 = gal.Dataset(*(t(a, d, dev) for a in (single.u, single.v, Vs.real + single.noise_re,
                                                Vs.imag + single.noise_im, single.w)))
    Is = t(single.I, d, dev)
    c2s = float(ds2.chi2Profile(Is, single.Rmin, single.dR, single.N, single.dxy, single.inc,
                                single.PA, single.dRA, single.dDec))

    def scene_jobs(scene, with_vis, first):
        # share indices count from the call's first job
        jobs = ds._scene_jobs(_gpu_sources(g, d, dev))
        for j in jobs:
            j["scene"] = scene
            if j["share"] is not None:
                j["share"] += first
        if with_vis:
            jobs[-1]["vis"] = torch.empty(ds.M, dtype=torch.complex128, device=dev)
        return jobs

    geo_s = torch.tensor([single.Rmin, single.dR, single.inc, single.PA, single.dRA, single.dDec],
                         dtype=torch.float64, device=dev)
    alone = {"ds": ds2, "kind": gal.JOB_PROFILE, "Nxy": single.N, "dxy": single.dxy, "model": Is,
             "geo": geo_s}
    A = scene_jobs(7, True, 1)
    B = scene_jobs(3, False, 2 + len(A))
    jobs = [alone] + A + [dict(alone)] + B
    grads = [None] * len(jobs)
    for k, j in enumerate(jobs[1:1 + len(A)], start=1):
        if j["model"] is not None:
            grads[k] = torch.empty_like(j["model"])
    c2 = gal.batch_exec(jobs, grads).cpu().numpy()
    assert c2[0] == c2[1 + len(A)]
    assert abs(c2[0] - c2s) <= 1e-12 * c2s
    for k in range(1, 1 + len(A)):
        assert abs(c2[k] - float(c2_alone)) <= 1e-12 * float(c2_alone)
    for k in range(2 + len(A), len(jobs)):
        assert c2[k] == c2[1]  # the same scene again, without gradients
    for k, gk in enumerate(grads[1:1 + len(A)]):
        if gk is None:
            assert g_alone[k] is None
            continue
        assert _rel(gk.cpu().numpy(), g_alone[k].cpu().numpy()) <= 1e-12, k
    assert_vis_close(A[-1]["vis"].cpu().numpy(), Vo, d, "vis in the mix")


def test_persistent_batch_of_fields_follows_updated_geometry():
    # a plan of four walkers, each a scene of the five sources; the geometry
    # tensors are rewritten between executions
    dev = device()
    gal = _gal()
    d = np.float64
    o, g, u, v, nre, nim, w = _field(5300, d, M=8000)
    Vo = oracle.sample_sources(o, u, v)
    ds = gal.Dataset(*(t(a, d, dev) for a in (u, v, Vo.real + nre, Vo.imag + nim, w)))
    jobs = []
    for walker in range(4):
        js = ds._scene_jobs(_gpu_sources(g, d, dev))
        for j in js:
            j["scene"] = walker + 1
            j["geo"][3] += 0.1 * walker
            if j["share"] is not None:
                j["share"] += 5 * walker
        jobs += js
    b = gal.Batch(jobs)
    info = b.info()
    assert info["sample_groups"] == 2  # 16 jobs per group at most: scenes of 5, 3 + 1
    for rep in range(2):
        c2 = b.chi2().cpu().numpy()
        for walker in range(4):
            geo = [jobs[5 * walker + k]["geo"].cpu().numpy() for k in range(5)]
            src = []
            for s, gg in zip(o, geo):
                s2 = dict(s, PA=gg[3], dRA=gg[4], dDec=gg[5])
                if s.get("share") is None:
                    s2["inc"] = gg[2]
                src.append(s2)
            Vw = oracle.sample_sources(src, u, v)
            c2o = oracle.chi2(Vw, Vo.real + nre, Vo.imag + nim, w)
            tol = chi2_bound(c2o, np.full(Vw.size, 1e-10 * np.max(np.abs(Vw))), w)
            for k in range(5):
                assert abs(c2[5 * walker + k] - c2o) <= tol, (rep, walker, k)
        for j in jobs:
            j["geo"][4] += 0.5 * g[1]["dxy"]
    b.close()


def test_uv_only_dataset_and_single_source_scene():
    # visibilities of a field on a dataset without observations (chi^2 = 0);
    # a one-source scene equals the source's own sampling call
    dev = device()
    gal = _gal()
    import torch

    d = np.float64
    o, g, u, v, *_ = _field(5400, d, M=5000)
    dsu = gal.Dataset(t(u, d, dev), t(v, d, dev))
    assert_vis_close(dsu.sampleSources(_gpu_sources(g, d, dev)).cpu().numpy(),
                     oracle.sample_sources(o, u, v), d, "uv-only field")
    assert float(dsu.chi2Sources(_gpu_sources(g, d, dev))) == 0.0
    src = _gpu_sources(g[:1], d, dev)
    V1 = dsu.sampleSources(src).cpu().numpy()
    s = g[0]
    Vs = dsu.sampleImage(src[0]["model"], s["dxy"], s["PA"], s["dRA"], s["dDec"], s["inc"])
    assert np.max(np.abs(V1 - Vs.cpu().numpy())) <= 1e-12 * np.max(np.abs(V1))
    with pytest.raises(gal.GalarioError):
        dsu.chi2Sources(_gpu_sources(g, d, dev), grad=True)  # no observations to fit
    del torch


def test_plan_rejects_bad_scenes():
    dev = device()
    gal = _gal()
    import torch

    d = np.float64
    o, g, u, v, nre, nim, w = _field(5500, d, M=2000)
    ds = gal.Dataset(*(t(a, d, dev) for a in (u, v, nre, nim, w)))
    ds2 = gal.Dataset(*(t(a, d, dev) for a in (u, v, nre, nim, w)))
    base = ds._scene_jobs(_gpu_sources(g, d, dev))

    def run(jobs, grads=None):
        with pytest.raises(gal.GalarioError):
            gal.batch_exec(jobs, grads)

    j = [dict(x) for x in base]
    j[2]["scene"] = 2  # shares a spectrum outside its scene
    run(j)
    j = [dict(x) for x in base]
    j[3]["share"] = 2  # shares from a sharer
    run(j)
    j = [dict(x) for x in base]
    j[2]["share"] = 0  # the owner is an image, the sharer a profile
    run(j)
    j = [dict(x) for x in base]
    j[4]["ds"] = ds2  # a scene over two datasets
    run(j)
    j = [dict(x) for x in base]
    j[2]["model"] = torch.zeros(7, dtype=torch.float64, device=dev)
    grads = [None] * len(j)
    grads[2] = torch.empty(7, dtype=torch.float64, device=dev)  # a sharer's own gradient
    run(j, grads)


def test_field_of_copies_2048_M1e6():
    # the full-size workload: a 2048^2 profile and 15 copies at other offsets
    # and orientations sharing its spectrum, M = 10^6; every visibility and
    # chi^2 against the oracle
    dev = device()
    gal = _gal()
    d = np.float64
    c = wl.profile_2048()
    src_o = wl.field_of_copies(c, 16, seed=5600)
    Vo = oracle.sample_sources(src_o, c.u, c.v)
    re, im = Vo.real + c.noise_re, Vo.imag + c.noise_im
    ds = gal.Dataset(*(t(a, d, dev) for a in (c.u, c.v, re, im, c.w)))
    I = t(c.I, d, dev)
    src_g = [{k: v for k, v in s.items() if k != "I"} for s in src_o]
    for s in src_g:
        s["model"] = I if s.get("share") is None else None
    Vg = ds.sampleSources(src_g).cpu().numpy()
    assert_vis_close(Vg, Vo, d, "16 copies 2048")
    c2o = oracle.chi2(Vo, re, im, c.w)
    c2g = float(ds.chi2Sources(src_g))
    assert abs(c2g - c2o) <= chi2_bound(c2o, Vg - Vo, c.w)
