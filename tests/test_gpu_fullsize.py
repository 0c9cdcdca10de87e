"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (device-resident dataset calls).

 - 256^2 chi2Image, M = 10^4: every output against the full oracle.
 - 2048^2 chi2Profile, M = 10^6 (the benchmark workload): every visibility
   and chi^2 against the full oracle (direct DFT, a few seconds on the host).
 - 4096^2 chi2Image, M = 5e6, FP64 and FP32: visibilities at sampled points
   against the oracle's per-node double sums; chi^2 against the host sum of
   the sampled model (a property that holds at any size).
 - 8192^2 (largest supported image): sampled points.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import assert_vis_close, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu


def _gal():
    import paper_1709_06999_amd as gal

    return gal


def test_gaussian_image_256_M1e4_full_oracle():
    dev = device()
    gal = _gal()
    c = wl.gaussian_image_256()
    d = np.float64
    kw = dict(PA=c.PA, dRA=c.dRA, dDec=c.dDec, inc=c.inc)
    Vo = oracle.sampleImage(c.image, c.dxy, c.u, c.v, **kw)
    re, im = Vo.real + c.noise_re, Vo.imag + c.noise_im
    c2o = oracle.chi2(Vo, re, im, c.w)
    img = t(c.image, d, dev)
    args = [t(a, d, dev) for a in (c.u, c.v, re, im, c.w)]
    c2g = float(gal.chi2Image(img, c.dxy, *args, **kw))
    Vg = gal.sampleImage(img, c.dxy, args[0], args[1], **kw).cpu().numpy()
    assert_vis_close(Vg, Vo, d, "gaussian 256 raw")
    assert abs(c2g - c2o) <= chi2_bound(c2o, Vg - Vo, c.w)
    ds = gal.Dataset(*args)
    c2d = float(ds.chi2Image(img, c.dxy, **kw))
    Vd = ds.sampleImage(img, c.dxy, **kw).cpu().numpy()
    assert_vis_close(Vd, Vo, d, "gaussian 256 dataset")
    assert abs(c2d - c2o) <= chi2_bound(c2o, Vd - Vo, c.w)
    # chi^2 at the noise level: E = 2M, sd = 2 sqrt(M)
    assert abs(c2o - 2 * c.M) < 6 * 2 * np.sqrt(c.M)


@pytest.fixture(scope="module")
def profile_2048_oracle():
    c = wl.profile_2048()
    Vo = oracle.sampleProfile(c.I, c.Rmin, c.dR, c.N, c.dxy, c.u, c.v, c.inc, c.PA, c.dRA, c.dDec)
    return c, Vo


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_profile_2048_M1e6_full_oracle(profile_2048_oracle, dtype):
    dev = device()
    gal = _gal()
    c, Vo64 = profile_2048_oracle
    if dtype == np.float32:
        Vo = oracle.sampleProfile(rounded(c.I, dtype), c.Rmin, c.dR, c.N, c.dxy,
                                  rounded(c.u, dtype), rounded(c.v, dtype), c.inc, c.PA, c.dRA,
                                  c.dDec)
    else:
        Vo = Vo64
    re = rounded(Vo.real + c.noise_re, dtype)
    im = rounded(Vo.imag + c.noise_im, dtype)
    w = rounded(c.w, dtype)
    ds = gal.Dataset(*(t(a, dtype, dev) for a in (c.u, c.v, re, im, w)))
    I = t(c.I, dtype, dev)
    kw = dict(inc=c.inc, PA=c.PA, dRA=c.dRA, dDec=c.dDec)
    Vd = ds.sampleProfile(I, c.Rmin, c.dR, c.N, c.dxy, **kw).cpu().numpy()
    err = assert_vis_close(Vd, Vo, dtype, "profile 2048")
    c2d = float(ds.chi2Profile(I, c.Rmin, c.dR, c.N, c.dxy, **kw))
    c2o = oracle.chi2(Vo, re, im, w)
    dV = np.abs(Vd - Vo) + (np.abs(Vd) * 2.0**-23 if dtype == np.float32 else 0.0)
    assert abs(c2d - c2o) <= chi2_bound(c2o, dV, w), (c2d, c2o)
    print(f"profile 2048 {np.dtype(dtype).name}: max|dV|/max|V| = {err:.3e}, chi2 gpu {c2d:.15g} "
          f"oracle {c2o:.15g}", flush=True)
    # the same through the raw-array call (full spectrum)
    c2r = float(gal.chi2Profile(I, c.Rmin, c.dR, c.N, c.dxy, *(t(a, dtype, dev) for a in
                                                              (c.u, c.v, re, im, w)), **kw))
    assert abs(c2r - c2o) <= chi2_bound(c2o, dV, w)
    ds.close()


@pytest.fixture(scope="module")
def blobs_4096_case():
    return wl.blobs_4096()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_blobs_4096_M5e6_sampled(blobs_4096_case, dtype):
    dev = device()
    gal = _gal()
    c = blobs_4096_case
    # observations: noise only (a full oracle model at 5e6 points is not needed
    # for parity; the model enters through V, checked point by point)
    re, im, w = rounded(c.noise_re, dtype), rounded(c.noise_im, dtype), rounded(c.w, dtype)
    args = [t(a, dtype, dev) for a in (c.u, c.v, re, im, w)]
    ds = gal.Dataset(*args)
    img = t(c.image, dtype, dev)
    Vd = ds.sampleImage(img, c.dxy, c.PA, c.dRA, c.dDec, c.inc).cpu().numpy()
    c2d = float(ds.chi2Image(img, c.dxy, c.PA, c.dRA, c.dDec, c.inc))
    # sampled points: the small-|uv| core, the largest radii and a uniform draw
    rng = np.random.default_rng(1203)
    rho = np.hypot(c.u, c.v)
    order = np.argsort(rho)
    idx = np.unique(np.concatenate([order[:24], order[-24:], rng.choice(c.M, 80, replace=False)]))
    Vo = oracle.sample_direct(rounded(c.image, dtype), c.dxy, rounded(c.u[idx], dtype),
                              rounded(c.v[idx], dtype), c.PA, c.dRA, c.dDec, c.inc)
    # tolerance relative to the total flux (= V at the origin, an upper bound of max|V|)
    flux = float(np.sum(rounded(c.image, dtype)))
    scale = max(np.max(np.abs(Vo)), flux)
    err = np.max(np.abs(Vd[idx] - Vo))
    tol = (1e-10 if dtype == np.float64 else 1e-4) * scale
    assert err <= tol, (err, tol)
    # chi^2 of the kernel equals the host sum over the sampled model
    c2h = oracle.chi2(Vd.astype(np.complex128), re, im, w)
    if dtype == np.float64:
        assert abs(c2d - c2h) <= 1e-11 * c2h
    else:
        assert abs(c2d - c2h) <= chi2_bound(c2h, np.abs(Vd) * 2.0**-23, w)
    ds.close()


def test_largest_image_8192_sampled():
    dev = device()
    gal = _gal()
    N, M = 8192, 50000
    case = wl.random_case(N, M, seed=8192)
    d = np.float64
    Vg = gal.sampleImage(t(case.image, d, dev), case.dxy, t(case.u, d, dev), t(case.v, d, dev),
                         case.PA, case.dRA, case.dDec, case.inc).cpu().numpy()
    idx = np.random.default_rng(1).choice(M, 12, replace=False)
    Vo = oracle.sample_direct(case.image, case.dxy, case.u[idx], case.v[idx], case.PA, case.dRA,
                              case.dDec, case.inc)
    scale = max(np.max(np.abs(Vo)), abs(np.sum(case.image)))
    assert np.max(np.abs(Vg[idx] - Vo)) <= 1e-10 * scale
