"""Every compiled FFT variant of every pass (rows of an image, columns, rows
and columns of a swept profile; for swept rows also the half-length transform
of even rows) against the oracle, in single calls and in a batch, at a small
and at the benchmark image size.  The variant in use is otherwise whatever
the autotuner picked, so each one is checked here."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import assert_vis_close, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,M,dtype", [(256, 20000, np.float64), (256, 20000, np.float32),
                                       (2048, 30000, np.float64)])
def test_every_variant_matches_oracle(N, M, dtype):
    dev = device()
    import torch

    import paper_1709_06999_amd as gal

    tdt = torch.float64 if dtype == np.float64 else torch.float32
    prof = wl.random_case(N, M, seed=3800 + N, kind="profile", fill=0.9)
    img = wl.random_case(N, 10, seed=3801 + N)
    I = rounded(prof.I, dtype)
    image = rounded(img.image, dtype)
    u, v = rounded(prof.u, dtype), rounded(prof.v, dtype)
    geo = dict(inc=prof.inc, PA=prof.PA, dRA=prof.dRA, dDec=prof.dDec)
    Vp = oracle.sampleProfile(I, prof.Rmin, prof.dR, N, prof.dxy, u, v, **geo)
    Vi = oracle.sampleImage(image, prof.dxy, u, v, geo["PA"], geo["dRA"], geo["dDec"], geo["inc"])
    re, im = rounded(Vp.real + prof.noise_re, dtype), rounded(Vp.imag + prof.noise_im, dtype)
    w = rounded(prof.w, dtype)
    c2o = oracle.chi2(Vp, re, im, w)
    ds = gal.Dataset(*(t(a, dtype, dev) for a in (u, v, re, im, w)))
    It, imt = t(I, dtype, dev), t(image, dtype, dev)
    geob = torch.tensor([[prof.Rmin, prof.dR, prof.inc, prof.PA + 0.1 * k, prof.dRA, prof.dDec]
                         for k in range(3)], dtype=torch.float64, device=dev)
    Ib = It.unsqueeze(0).repeat(3, 1).contiguous()
    try:
        for var in range(3):
            gal.tune_set(N, [var] * 4, tdt)
            what = f"N={N} {dtype.__name__} variant {var}"
            Vg = ds.sampleProfile(It, prof.Rmin, prof.dR, N, prof.dxy, **geo).cpu().numpy()
            assert_vis_close(Vg, Vp, dtype, what + " profile")
            assert_vis_close(ds.sampleImage(imt, prof.dxy, geo["PA"], geo["dRA"], geo["dDec"],
                                            geo["inc"]).cpu().numpy(), Vi, dtype, what + " image")
            b = gal.profile_batch(ds, Ib, geob, N, prof.dxy)
            c2b = b.chi2().cpu().numpy()
            b.close()
            c2s = float(ds.chi2Profile(It, prof.Rmin, prof.dR, N, prof.dxy, **geo))
            tol = 1e-12 if dtype == np.float64 else 1e-6
            assert abs(c2b[0] - c2s) <= tol * c2s, (what, c2b[0], c2s)
            # chi^2 within the bound of this variant's model error (plus the
            # FP32 rounding of the model it accumulates)
            dV = np.abs(Vg - Vp) + (np.abs(Vg) * 2.0 ** -23 if dtype == np.float32 else 0.0)
            assert abs(c2s - c2o) <= chi2_bound(c2o, dV, w), (what, c2s, c2o)
    finally:
        gal.tune_set(N, [-1] * 4, tdt)
        ds.close()


def test_every_variant_at_the_largest_image():
    # 8192^2 (the largest size), FP64 profile: every variant against the
    # oracle's direct double sums at sampled points (tolerance relative to the
    # total flux, |V(0, 0)|), the variants against each other at every point,
    # and the batch against the single call
    dev = device()
    import torch

    import paper_1709_06999_amd as gal

    N, d = 8192, np.float64
    c = wl.random_case(N, 20000, seed=3901, kind="profile", fill=0.9)
    geo = dict(inc=c.inc, PA=c.PA, dRA=c.dRA, dDec=c.dDec)
    img = oracle.sweep(c.I, c.Rmin, c.dR, N, c.dxy, c.inc)
    flux = float(np.sum(img))
    pick = np.random.default_rng(3902).choice(c.M, 8, replace=False)
    Vo = oracle.sample_direct(img, c.dxy, c.u[pick], c.v[pick], c.PA, c.dRA, c.dDec, 0.0)
    del img
    ds = gal.Dataset(*(t(a, d, dev) for a in (c.u, c.v, c.noise_re, c.noise_im, c.w)))
    It = t(c.I, d, dev)
    geob = torch.tensor([[c.Rmin, c.dR, c.inc, c.PA, c.dRA, c.dDec]] * 2, dtype=torch.float64,
                        device=dev)
    Ib = It.unsqueeze(0).repeat(2, 1).contiguous()
    ref = None
    try:
        for var in range(3):
            gal.tune_set(N, [var] * 4, torch.float64)
            Vg = ds.sampleProfile(It, c.Rmin, c.dR, N, c.dxy, **geo).cpu().numpy()
            err = np.max(np.abs(Vg[pick] - Vo)) / flux
            assert err <= 1e-10, (var, err)
            if ref is None:
                ref = Vg
            assert np.max(np.abs(Vg - ref)) <= 1e-12 * flux, var
            b = gal.profile_batch(ds, Ib, geob, N, c.dxy)
            c2b = b.chi2().cpu().numpy()
            b.close()
            c2s = float(ds.chi2Profile(It, c.Rmin, c.dR, N, c.dxy, **geo))
            assert abs(c2b[0] - c2s) <= 1e-12 * c2s and c2b[0] == c2b[1], var
    finally:
        gal.tune_set(N, [-1] * 4, torch.float64)
        ds.close()
