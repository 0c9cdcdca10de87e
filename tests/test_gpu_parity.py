"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Sizes here run the oracle in seconds yet span several FFT tiles, ragged
point counts (not multiples of the 1024-point sample block) and both
precisions.  Tolerances: |V_gpu - V_oracle| <= 1e-10 max|V| (FP64) and
1e-4 max|V| (FP32, oracle fed the FP32-rounded inputs); chi^2 within the
Cauchy-Schwarz bound of the measured model error.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import assert_vis_close, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu

DTYPES = [np.float64, np.float32]


def _gal():
    import paper_1709_06999_amd as gal

    return gal


def _oracle_V(case, dtype, kind=None):
    kind = kind or case.kind
    u, v = rounded(case.u, dtype), rounded(case.v, dtype)
    if kind == "image":
        return oracle.sampleImage(rounded(case.image, dtype), case.dxy, u, v, case.PA, case.dRA,
                                  case.dDec, case.inc)
    return oracle.sampleProfile(rounded(case.I, dtype), case.Rmin, case.dR, case.N, case.dxy, u, v,
                                case.inc, case.PA, case.dRA, case.dDec)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 32, 64, 128, 256, 512, 1024])
def test_spectrum_matches_oracle_grid(N, dtype):
    dev = device()
    gal = _gal()
    rng = np.random.default_rng(N)
    img = rng.normal(size=(N, N))
    G = gal.spectrum(t(img, dtype, dev)).cpu().numpy()
    Go = oracle.grid(rounded(img, dtype))
    scale = np.max(np.abs(Go))
    err = np.max(np.abs(G - Go))
    tol = (1e-12 if dtype == np.float64 else 2e-5) * scale
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 64, 256])
def test_sampler_on_oracle_spectrum(N, dtype):
    # the sampling kernel alone, fed the oracle's half spectrum
    dev = device()
    gal = _gal()
    case = wl.random_case(N, 3001, seed=200 + N)
    Go = oracle.grid(rounded(case.image, dtype))
    Gd = Go.astype(np.complex128 if dtype == np.float64 else np.complex64)
    import torch

    spec = torch.as_tensor(Gd, device=dev)
    Vg = gal.sample_spectrum(spec, case.dxy, t(case.u, dtype, dev), t(case.v, dtype, dev),
                             case.PA, case.dRA, case.dDec, case.inc).cpu().numpy()
    Vo = oracle.sample_grid(Gd.astype(np.complex128), N, case.dxy, rounded(case.u, dtype),
                            rounded(case.v, dtype), case.PA, case.dRA, case.dDec, case.inc)
    assert_vis_close(Vg, Vo, dtype, "sample_spectrum")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 64, 256])
def test_sweep_matches_oracle(N, dtype):
    dev = device()
    gal = _gal()
    case = wl.random_case(N, 10, seed=300 + N, kind="profile")
    img = gal.sweep(t(case.I, dtype, dev), case.Rmin, case.dR, N, case.dxy,
                    case.inc).cpu().numpy()
    ref = oracle.sweep(rounded(case.I, dtype), case.Rmin, case.dR, N, case.dxy, case.inc)
    tol = (1e-13 if dtype == np.float64 else 1e-6) * np.max(np.abs(ref))
    assert np.max(np.abs(img - ref)) <= tol


CASES = [(16, 1), (32, 777), (64, 1024), (128, 5003), (256, 20001), (512, 65537), (1024, 30000)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["image", "profile"])
@pytest.mark.parametrize("N,M", CASES)
def test_sample_parity(N, M, kind, dtype):
    dev = device()
    gal = _gal()
    case = wl.random_case(N, M, seed=N + 7 * M, kind=kind)
    u, v = t(case.u, dtype, dev), t(case.v, dtype, dev)
    if kind == "image":
        Vg = gal.sampleImage(t(case.image, dtype, dev), case.dxy, u, v, case.PA, case.dRA,
                             case.dDec, case.inc)
    else:
        Vg = gal.sampleProfile(t(case.I, dtype, dev), case.Rmin, case.dR, N, case.dxy, u, v,
                               case.inc, case.PA, case.dRA, case.dDec)
    Vo = _oracle_V(case, dtype)
    assert_vis_close(Vg.cpu().numpy(), Vo, dtype, f"{kind} N={N} M={M}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["image", "profile"])
@pytest.mark.parametrize("N,M", CASES)
def test_chi2_parity(N, M, kind, dtype):
    dev = device()
    gal = _gal()
    case = wl.random_case(N, M, seed=N + 7 * M + 1, kind=kind)
    Vo = _oracle_V(case, dtype)
    re = rounded(Vo.real + case.noise_re, dtype)
    im = rounded(Vo.imag + case.noise_im, dtype)
    w = rounded(case.w, dtype)
    args = [t(case.u, dtype, dev), t(case.v, dtype, dev), t(re, dtype, dev), t(im, dtype, dev),
            t(w, dtype, dev)]
    if kind == "image":
        img = t(case.image, dtype, dev)
        c2g = float(gal.chi2Image(img, case.dxy, *args, case.PA, case.dRA, case.dDec, case.inc))
        Vg = gal.sampleImage(img, case.dxy, args[0], args[1], case.PA, case.dRA, case.dDec,
                             case.inc).cpu().numpy()
    else:
        I = t(case.I, dtype, dev)
        c2g = float(gal.chi2Profile(I, case.Rmin, case.dR, N, case.dxy, *args, case.inc, case.PA,
                                    case.dRA, case.dDec))
        Vg = gal.sampleProfile(I, case.Rmin, case.dR, N, case.dxy, args[0], args[1], case.inc,
                               case.PA, case.dRA, case.dDec).cpu().numpy()
    c2o = oracle.chi2(Vo, re, im, w)
    dV = np.abs(Vg - Vo)
    if dtype == np.float32:
        dV = dV + np.abs(Vg) * 2.0**-23   # the chi^2 kernel uses V before rounding to float
    bound = chi2_bound(c2o, dV, w)
    assert abs(c2g - c2o) <= bound, (c2g, c2o, bound)
    # the chi^2 kernel and the sample kernel agree on the model (in FP32 the
    # sample output is V rounded to float; the chi^2 kernel uses V unrounded)
    c2s = oracle.chi2(Vg.astype(np.complex128), re, im, w)
    if dtype == np.float64:
        assert abs(c2g - c2s) <= 1e-11 * c2s + 1e-300
    else:
        assert abs(c2g - c2s) <= chi2_bound(c2s, np.abs(Vg) * 2.0**-23, w)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["image", "profile"])
def test_dataset_path_matches_raw_path_and_oracle(kind, dtype):
    dev = device()
    gal = _gal()
    N, M = 256, 12345
    case = wl.random_case(N, M, seed=404, kind=kind, fill=0.6)
    Vo = _oracle_V(case, dtype)
    re = rounded(Vo.real + case.noise_re, dtype)
    im = rounded(Vo.imag + case.noise_im, dtype)
    w = rounded(case.w, dtype)
    u, v = t(case.u, dtype, dev), t(case.v, dtype, dev)
    ds = gal.Dataset(u, v, t(re, dtype, dev), t(im, dtype, dev), t(w, dtype, dev))
    assert abs(ds.rho_max - np.max(np.hypot(rounded(case.u, dtype), rounded(case.v, dtype)))) \
        <= 1e-12 * ds.rho_max
    if kind == "image":
        img = t(case.image, dtype, dev)
        Vd = ds.sampleImage(img, case.dxy, case.PA, case.dRA, case.dDec, case.inc).cpu().numpy()
        Vr = gal.sampleImage(img, case.dxy, u, v, case.PA, case.dRA, case.dDec,
                             case.inc).cpu().numpy()
        c2d = float(ds.chi2Image(img, case.dxy, case.PA, case.dRA, case.dDec, case.inc))
    else:
        I = t(case.I, dtype, dev)
        Vd = ds.sampleProfile(I, case.Rmin, case.dR, N, case.dxy, case.inc, case.PA, case.dRA,
                              case.dDec).cpu().numpy()
        Vr = gal.sampleProfile(I, case.Rmin, case.dR, N, case.dxy, u, v, case.inc, case.PA,
                               case.dRA, case.dDec).cpu().numpy()
        c2d = float(ds.chi2Profile(I, case.Rmin, case.dR, N, case.dxy, case.inc, case.PA,
                                   case.dRA, case.dDec))
    # pruning the spectrum does not change the samples (same FFT arithmetic per node)
    assert np.array_equal(Vd, Vr)
    assert_vis_close(Vd, Vo, dtype, "dataset")
    c2o = oracle.chi2(Vo, re, im, w)
    dV = np.abs(Vd - Vo) + (np.abs(Vd) * 2.0**-23 if dtype == np.float32 else 0.0)
    assert abs(c2d - c2o) <= chi2_bound(c2o, dV, w)
    ds.close()


def test_profile_equals_image_of_sweep():
    # sampleProfile == sampleImage(sweep(I)) to rounding (Sec. 5: identical to machine precision)
    dev = device()
    gal = _gal()
    case = wl.random_case(512, 4000, seed=505, kind="profile")
    I = t(case.I, np.float64, dev)
    u, v = t(case.u, np.float64, dev), t(case.v, np.float64, dev)
    img = gal.sweep(I, case.Rmin, case.dR, 512, case.dxy, case.inc)
    V1 = gal.sampleProfile(I, case.Rmin, case.dR, 512, case.dxy, u, v, case.inc, case.PA,
                           case.dRA, case.dDec).cpu().numpy()
    V2 = gal.sampleImage(img, case.dxy, u, v, case.PA, case.dRA, case.dDec).cpu().numpy()
    assert np.max(np.abs(V1 - V2)) <= 1e-13 * np.max(np.abs(V1))


def test_chi2_is_bitwise_repeatable():
    dev = device()
    gal = _gal()
    case = wl.random_case(256, 200003, seed=606)
    d = np.float64
    args = [t(a, d, dev) for a in (case.u, case.v, case.noise_re, case.noise_im, case.w)]
    img = t(case.image, d, dev)
    vals = {float(gal.chi2Image(img, case.dxy, *args, case.PA, case.dRA, case.dDec, case.inc))
            for _ in range(5)}
    assert len(vals) == 1


# ---------------------------------------------------------------------------
# edge cases and errors
def test_empty_and_single_point():
    dev = device()
    gal = _gal()
    import torch

    img = t(np.random.default_rng(1).normal(size=(64, 64)), np.float64, dev)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    assert float(gal.chi2Image(img, 1e-7, e, e, e, e, e)) == 0.0
    assert gal.sampleImage(img, 1e-7, e, e).numel() == 0
    case = wl.random_case(64, 1, seed=9)
    Vg = gal.sampleImage(t(case.image, np.float64, dev), case.dxy, t(case.u, np.float64, dev),
                         t(case.v, np.float64, dev), case.PA, case.dRA, case.dDec, case.inc)
    Vo = _oracle_V(case, np.float64)
    assert_vis_close(Vg.cpu().numpy(), Vo, np.float64, "M=1")


def test_off_grid_points_are_flagged_nan():
    dev = device()
    gal = _gal()
    N, dxy = 32, 1e-7
    du = 1.0 / (N * dxy)
    rng = np.random.default_rng(3)
    img = rng.normal(size=(N, N))
    u = np.array([0.5, N / 2 - 0.5, 0.0, 0.0, N / 2 + 0.2, 0.0, 3.2]) * du
    v = np.array([0.5, 0.0, N / 2 - 1.5, -(N / 2 - 0.25), 0.0, N / 2 - 0.5, -(N / 2 + 0.3)]) * du
    assert gal.read_status() == 0
    Vg = gal.sampleImage(t(img, np.float64, dev), dxy, t(u, np.float64, dev),
                         t(v, np.float64, dev)).cpu().numpy()
    Vo = oracle.sampleImage(img, dxy, u, v)
    assert np.array_equal(np.isnan(Vg), np.isnan(Vo))
    assert np.all(np.isnan(Vg[4:])) and np.all(np.isfinite(Vg[:4]))
    assert_vis_close(Vg[:4], Vo[:4], np.float64, "valid edge points")
    assert gal.read_status() == 1
    assert gal.read_status() == 0


# (u', v') in grid units and whether the stencil lies inside the spectrum
# (App. D: lower v' node in [-N/2, N/2 - 2] on the mirrored point, lower u'
# node <= N/2 - 1), for N = 32
PROFILE_EDGE_POINTS = [
    ((0.0, -1.0), True), ((0.0, -3.0), True), ((2.5, -15.0), True), ((1.0, -16.0), True),
    ((0.0, 14.5), True), ((-3.0, 2.0), True), ((-3.0, 16.0), True), ((15.5, 0.0), True),
    ((0.0, 0.0), True), ((-2.25, -7.0), True),
    ((3.0, -16.5), False), ((3.0, 15.0), False), ((-3.0, -15.0), False), ((16.0, 0.0), False),
    ((-16.0, 1.0), False),
]


@pytest.mark.parametrize("dtype", DTYPES)
def test_profile_edge_points_match_oracle(dtype):
    # swept profiles are sampled from their real, even spectrum; points on node
    # lines, on the validity limits and on both sides of the mirror, at exact
    # grid coordinates (N dxy = 2^-20, PA = 0), against the oracle's App. D
    # rule and values
    dev = device()
    gal = _gal()
    import torch

    # the status flag lives in the workspace of the call's precision
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    status = lambda: gal.read_status(tdt)
    N, dxy = 32, 2.0 ** -25
    du = 1.0 / (N * dxy)
    pts = np.array([p for p, _ in PROFILE_EDGE_POINTS])
    ok = np.array([k for _, k in PROFILE_EDGE_POINTS])
    u, v = pts[:, 0] * du, pts[:, 1] * du
    r = np.linspace(0.0, 1.0, 64)
    I = rounded((1.0 + 3.0 * np.exp(-(r / 0.3) ** 2)) / dxy ** 2, dtype)
    Rmin, dR, inc = 0.0, 1.2 * N * dxy / 63, 0.4
    Vo = oracle.sampleProfile(I, Rmin, dR, N, dxy, u, v, inc)
    assert np.array_equal(np.isfinite(Vo), ok)
    assert status() == 0
    Vg = gal.sampleProfile(t(I, dtype, dev), Rmin, dR, N, dxy, t(u, dtype, dev), t(v, dtype, dev),
                           inc).cpu().numpy()
    assert np.array_equal(np.isfinite(Vg), ok)
    assert_vis_close(Vg[ok], Vo[ok], dtype, "profile edge points")
    assert status() == 1
    # chi^2 over the valid points, then with the invalid ones: NaN and flagged
    rng = np.random.default_rng(11)
    re, im, w = rng.normal(size=u.size), rng.normal(size=u.size), rng.uniform(0.5, 1.5, u.size)
    args = [t(a[ok], dtype, dev) for a in (u, v, re, im, w)]
    c2g = float(gal.chi2Profile(t(I, dtype, dev), Rmin, dR, N, dxy, *args, inc))
    c2o = oracle.chi2(Vo[ok], *(rounded(a[ok], dtype) for a in (re, im, w)))
    dV = np.abs(Vg[ok] - Vo[ok]) + np.abs(Vo[ok]) * np.finfo(dtype).eps
    assert abs(c2g - c2o) <= chi2_bound(c2o, dV, rounded(w[ok], dtype)), (c2g, c2o)
    assert status() == 0
    c2n = float(gal.chi2Profile(t(I, dtype, dev), Rmin, dR, N, dxy,
                                *(t(a, dtype, dev) for a in (u, v, re, im, w)), inc))
    assert np.isnan(c2n)
    assert status() == 1
    # the valid points within the radius a dataset accepts (rho <= (N/2 - 1) du,
    # checked on the host) as a resident dataset: its own call and a one-job batch
    inr = ok & (np.hypot(u, v) <= (N / 2 - 1) * du)
    assert inr.sum() >= 5
    ds = gal.Dataset(*(t(a[inr], dtype, dev) for a in (u, v, re, im, w)))
    It = t(I, dtype, dev)
    c2o = oracle.chi2(Vo[inr], *(rounded(a[inr], dtype) for a in (re, im, w)))
    dV = np.abs(Vg[inr] - Vo[inr]) + np.abs(Vo[inr]) * np.finfo(dtype).eps
    c2d = float(ds.chi2Profile(It, Rmin, dR, N, dxy, inc, 0.0, 0.0, 0.0))
    geo = torch.tensor([Rmin, dR, inc, 0.0, 0.0, 0.0], dtype=torch.float64, device=dev)
    b = gal.Batch([{"ds": ds, "kind": gal.JOB_PROFILE, "Nxy": N, "dxy": dxy, "model": It,
                    "geo": geo}])
    c2b = float(b.chi2().cpu()[0])
    b.close()
    ds.close()
    for c in (c2d, c2b):
        assert abs(c - c2o) <= chi2_bound(c2o, dV, rounded(w[inr], dtype)), (c, c2o)
    assert status() == 0


def test_host_side_errors():
    dev = device()
    gal = _gal()
    from paper_1709_06999_amd import GalarioError

    img = t(np.zeros((56, 56)), np.float64, dev)
    u = t(np.zeros(4), np.float64, dev)
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        gal.sampleImage(img, 1e-7, u, u)                         # 56 = 2^3 7
    img = t(np.zeros((64, 64)), np.float64, dev)
    with pytest.raises(GalarioError, match="GAL_ERR_SCALAR"):
        gal.sampleImage(img, -1e-7, u, u)                        # dxy <= 0
    with pytest.raises(GalarioError, match="GAL_ERR_SCALAR"):
        gal.sampleImage(img, 1e-7, u, u, inc=1.6)                # cos(inc) < 0
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        gal.sampleProfile(t(np.ones(1), np.float64, dev), 0.0, 1e-7, 64, 1e-7, u, u)   # Nr < 2
    # workspace smaller than gal_workspace_bytes: rejected through the C ABI
    import ctypes
    import torch
    from paper_1709_06999_amd import _native

    small = torch.zeros(512, dtype=torch.uint8, device=dev)
    out = torch.empty(8, dtype=torch.float64, device=dev)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    rc = _native.lib().gal_sampleImage_d(p(img), 64, 1e-7, p(u), p(u), 4, 0.0, 0.0, 0.0, 0.0,
                                         p(out), p(small), 512, None)
    assert rc == -5
    rc = _native.lib().gal_sampleImage_d(None, 64, 1e-7, p(u), p(u), 4, 0.0, 0.0, 0.0, 0.0,
                                         p(out), p(small), 512, None)
    assert rc == -1
    # dataset reaching outside the spectrum: rejected before any launch
    N, dxy = 64, 1e-7
    du = 1.0 / (N * dxy)
    uu = t(np.array([0.0, (N / 2 - 0.9) * du]), np.float64, dev)
    ds = gal.Dataset(uu, uu * 0, uu * 0, uu * 0, uu * 0 + 1)
    with pytest.raises(GalarioError, match="GAL_ERR_UV_RANGE"):
        ds.chi2Image(img, dxy)
    ds.close()


def test_library_symbols_resolve_on_gpu():
    gal = _gal()
    from paper_1709_06999_amd import _native

    L = _native.lib()
    for n in _native.exported_names():
        assert hasattr(L, n), n
    assert "gfx950" in gal.version()
