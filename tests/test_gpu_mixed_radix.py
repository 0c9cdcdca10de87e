"""GPU parity at image sizes N = 2^a 3^b 5^c that are not powers of two (the
mixed-radix path: Stockham passes of radix 4, 2, 3 and 5).  Every visibility
against the full oracle (direct DFT) at 1e-10 (FP64) / 1e-4 (FP32) of
max|V|, chi^2 of a dataset against the oracle's within the Cauchy-Schwarz
bound, for images and swept profiles."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import assert_vis_close, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu

SIZES = [18, 48, 96, 160, 240, 480, 1000, 1536]
DTYPES = [np.float64, np.float32]


def _gal():
    import paper_1709_06999_amd as gal

    return gal


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["image", "profile"])
@pytest.mark.parametrize("N", SIZES)
def test_mixed_radix_against_oracle(N, kind, dtype):
    dev = device()
    gal = _gal()
    M = 2000
    c = wl.random_case(N, M, seed=7000 + N + (kind == "profile"), kind=kind)
    print(f"mixed radix N={N} {kind} {np.dtype(dtype).name}", flush=True)
    u, v = rounded(c.u, dtype), rounded(c.v, dtype)
    if kind == "image":
        Vo = oracle.sampleImage(rounded(c.image, dtype), c.dxy, u, v, c.PA, c.dRA, c.dDec, c.inc)
        model = t(c.image, dtype, dev)
        Vg = gal.sampleImage(model, c.dxy, t(c.u, dtype, dev), t(c.v, dtype, dev), c.PA, c.dRA,
                             c.dDec, c.inc)
    else:
        Vo = oracle.sampleProfile(rounded(c.I, dtype), c.Rmin, c.dR, N, c.dxy, u, v, c.inc, c.PA,
                                  c.dRA, c.dDec)
        model = t(c.I, dtype, dev)
        Vg = gal.sampleProfile(model, c.Rmin, c.dR, N, c.dxy, t(c.u, dtype, dev),
                               t(c.v, dtype, dev), c.inc, c.PA, c.dRA, c.dDec)
    Vg = Vg.cpu().numpy()
    assert_vis_close(Vg, Vo, dtype, f"N={N} {kind}")
    # chi^2 on a resident dataset (pruned spectrum, locality order)
    re, im, w = (rounded(a, dtype) for a in (Vo.real + c.noise_re, Vo.imag + c.noise_im, c.w))
    ds = gal.Dataset(*(t(a, dtype, dev) for a in (c.u, c.v, re, im, w)))
    if kind == "image":
        c2g = float(ds.chi2Image(model, c.dxy, c.PA, c.dRA, c.dDec, c.inc))
    else:
        c2g = float(ds.chi2Profile(model, c.Rmin, c.dR, N, c.dxy, c.inc, c.PA, c.dRA, c.dDec))
    ds.close()
    c2o = oracle.chi2(Vo, re, im, w)
    dV = np.abs(Vg - Vo) + np.abs(Vo) * np.finfo(dtype).eps
    assert abs(c2g - c2o) <= chi2_bound(c2o, dV, w), (c2g, c2o)


def test_mixed_radix_sizes_refused_elsewhere():
    dev = device()
    gal = _gal()
    from paper_1709_06999_amd import GalarioError

    c = wl.random_case(48, 100, seed=11, kind="image")
    d = np.float64
    img = t(c.image, d, dev)
    u, v = t(c.u, d, dev), t(c.v, d, dev)
    # 7 is not a factor the path takes; 50 = 2 * 5^2 is
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        gal.sampleImage(t(np.zeros((56, 56)), d, dev), c.dxy, u, v)
    gal.sampleImage(t(np.zeros((50, 50)), d, dev), c.dxy, u, v)
    # gradients and the separate spectrum call stay on powers of two
    ds = gal.Dataset(u, v, t(c.noise_re, d, dev), t(c.noise_im, d, dev), t(c.w, d, dev))
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        ds.chi2Image_grad(img, c.dxy, c.PA)
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        gal.spectrum(img)
    ds.close()
