"""GPU chi^2 gradient with respect to the geometry (PA, dRA, dDec, inc)
against the oracle's chain rule, against central differences of the GPU
chi^2, in FP32, and at the full profile workload (2048^2, M = 10^6)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import device, rounded, t

pytestmark = pytest.mark.gpu

NAMES = ("PA", "dRA", "dDec", "inc")


def _gal():
    import paper_1709_06999_amd as gal

    return gal


def _obs(case, rng, offset=0.05):
    if case.kind == "image":
        Vo = oracle.sampleImage(case.image, case.dxy, case.u, case.v, case.PA, case.dRA,
                                case.dDec, 0.3)
    else:
        Vo = oracle.sampleProfile(case.I, case.Rmin, case.dR, case.N, case.dxy, case.u, case.v,
                                  0.3, case.PA, case.dRA, case.dDec)
    # observations of a slightly different source, so that no derivative vanishes
    return ((1.0 + offset) * Vo.real + case.noise_re, (1.0 - offset) * Vo.imag + case.noise_im,
            rng.uniform(0.5, 2.0, case.M))


def _scale(c2, dxy):
    # natural magnitudes of the four derivatives (chi^2 per radian of PA and
    # inc, per pixel size of the offsets)
    return np.array([c2, c2 / dxy, c2 / dxy, c2])


@pytest.mark.parametrize("kind", ["image", "profile"])
@pytest.mark.parametrize("N,M", [(16, 500), (64, 6001), (256, 30011)])
def test_geograd_matches_oracle(kind, N, M):
    dev = device()
    gal = _gal()
    d = np.float64
    case = wl.random_case(N, M, seed=4000 + N, kind=kind, Nr=60, fill=0.8)
    rng = np.random.default_rng(4100 + N)
    re, im, w = _obs(case, rng)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=0.35)
    ds = gal.Dataset(*(t(a, d, dev) for a in (case.u, case.v, re, im, w)))
    if kind == "image":
        c2o, go = oracle.geograd_image(case.image, case.dxy, case.u, case.v, re, im, w, **kw)
        c2g, gg = ds.chi2Image_geograd(t(case.image, d, dev), case.dxy, **kw)
    else:
        c2o, go = oracle.geograd_profile(case.I, case.Rmin, case.dR, N, case.dxy, case.u,
                                         case.v, re, im, w, **kw)
        c2g, gg = ds.chi2Profile_geograd(t(case.I, d, dev), case.Rmin, case.dR, N, case.dxy,
                                         **kw)
    gg = gg.cpu().numpy()
    assert abs(float(c2g) - c2o) <= 1e-10 * c2o
    tol = 1e-9 * _scale(c2o, case.dxy) + 1e-8 * np.abs(go)
    assert np.all(np.abs(gg - go) <= tol), list(zip(NAMES, gg, go, tol))


@pytest.mark.parametrize("kind", ["image", "profile"])
def test_geograd_central_differences_on_gpu(kind):
    dev = device()
    gal = _gal()
    d = np.float64
    # few enough points, and a step small enough, that no point crosses a cell
    # edge or the mirror line (the bilinear interpolant's derivative jumps there)
    case = wl.random_case(64, 3000, seed=4200 + (kind == "profile"), kind=kind, Nr=80, fill=0.7)
    rng = np.random.default_rng(4210)
    re, im, w = _obs(case, rng, offset=0.2)
    ds = gal.Dataset(*(t(a, d, dev) for a in (case.u, case.v, re, im, w)))
    base = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=0.35)
    if kind == "image":
        img = t(case.image, d, dev)
        f = lambda **kw: float(ds.chi2Image(img, case.dxy, **kw))
        c2, g = ds.chi2Image_geograd(img, case.dxy, **base)
    else:
        I = t(case.I, d, dev)
        f = lambda **kw: float(ds.chi2Profile(I, case.Rmin, case.dR, 64, case.dxy, **kw))
        c2, g = ds.chi2Profile_geograd(I, case.Rmin, case.dR, 64, case.dxy, **base)
    g = g.cpu().numpy()
    steps = {"PA": 1e-7, "dRA": 1e-4 * case.dxy, "dDec": 1e-4 * case.dxy, "inc": 1e-7}
    for k, name in enumerate(NAMES):
        hi, lo = dict(base), dict(base)
        hi[name] += steps[name]
        lo[name] -= steps[name]
        fd = (f(**hi) - f(**lo)) / (2 * steps[name])
        assert abs(g[k] - fd) <= 1e-4 * max(abs(fd), 1e-3 * _scale(float(c2), case.dxy)[k]), \
            (name, g[k], fd)


@pytest.mark.parametrize("kind", ["image", "profile"])
def test_geograd_fp32_close_to_fp64_oracle(kind):
    dev = device()
    gal = _gal()
    f = np.float32
    case = wl.random_case(128, 10000, seed=4300 + (kind == "profile"), kind=kind, Nr=100)
    rng = np.random.default_rng(4310)
    re, im, w = _obs(case, rng, offset=0.3)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=0.35)
    ds = gal.Dataset(*(t(a, f, dev) for a in (case.u, case.v, re, im, w)))
    args = [rounded(a, f) for a in (case.u, case.v, re, im, w)]
    if kind == "image":
        c2o, go = oracle.geograd_image(rounded(case.image, f), case.dxy, *args, **kw)
        _, gg = ds.chi2Image_geograd(t(case.image, f, dev), case.dxy, **kw)
    else:
        c2o, go = oracle.geograd_profile(rounded(case.I, f), case.Rmin, case.dR, 128, case.dxy,
                                         *args, **kw)
        _, gg = ds.chi2Profile_geograd(t(case.I, f, dev), case.Rmin, case.dR, 128, case.dxy, **kw)
    gg = gg.cpu().numpy()
    tol = 1e-4 * _scale(c2o, case.dxy) + 1e-3 * np.abs(go)
    assert np.all(np.abs(gg - go) <= tol), list(zip(NAMES, gg, go, tol))


def test_geograd_profile_2048_full_size():
    dev = device()
    gal = _gal()
    d = np.float64
    c = wl.profile_2048()
    rng = np.random.default_rng(4400)
    Vo = oracle.sampleProfile(c.I, c.Rmin, c.dR, c.N, c.dxy, c.u, c.v, c.inc, c.PA, c.dRA, c.dDec)
    re, im, w = 1.02 * Vo.real + c.noise_re, Vo.imag + c.noise_im, c.w
    kw = dict(inc=c.inc, PA=c.PA, dRA=c.dRA + 0.3 * c.dxy, dDec=c.dDec - 0.2 * c.dxy)
    c2o, go = oracle.geograd_profile(c.I, c.Rmin, c.dR, c.N, c.dxy, c.u, c.v, re, im, w, **kw)
    ds = gal.Dataset(*(t(a, d, dev) for a in (c.u, c.v, re, im, w)))
    c2g, gg = ds.chi2Profile_geograd(t(c.I, d, dev), c.Rmin, c.dR, c.N, c.dxy, **kw)
    gg = gg.cpu().numpy()
    print(f"geograd 2048: gpu {gg}, oracle {go}", flush=True)
    assert abs(float(c2g) - c2o) <= 1e-10 * c2o
    tol = 1e-9 * _scale(c2o, c.dxy) + 1e-8 * np.abs(go)
    assert np.all(np.abs(gg - go) <= tol), list(zip(NAMES, gg, go, tol))
