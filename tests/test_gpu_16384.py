"""GPU parity at 16384^2, the largest image of the paper's timing tables
(Sec. 6.1 Table tb:timings.chi2Profile, App. B Table tb:timings.chi2Image).

At this size a full-length FP64 column (256 KB) does not fit in a
workgroup's LDS: swept profiles take the half-length transform of even
sequences in both passes, images take the two-launch (four-step) column pass
in FP64 and the in-LDS one in FP32.  Checked against the oracle's direct
double sums on sampled points, and chi^2 on a dataset of those points against
the oracle's chi^2 of the same model within the Cauchy-Schwarz bound."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL_V, chi2_bound, device, rounded, t

pytestmark = pytest.mark.gpu

N = 16384
M = 20000
NS = 12   # sampled points


def _gal():
    import paper_1709_06999_amd as gal

    return gal


@pytest.fixture(scope="module", params=["profile", "image"])
def case16k(request):
    """The case and, per precision, the oracle's samples of the inputs as the
    GPU sees them (FP32: model and uv coordinates rounded to float)."""
    kind = request.param
    c = wl.random_case(N, M, seed=16384 + (kind == "image"), kind=kind)
    idx = np.sort(np.random.default_rng(3).choice(M, NS, replace=False))
    inc = c.inc if kind == "image" else 0.0   # a profile's inclination is in its sweep
    ref = {}
    for d in (np.float64, np.float32):
        img = (rounded(c.image, d) if kind == "image"
               else oracle.sweep(rounded(c.I, d), c.Rmin, c.dR, N, c.dxy, c.inc))
        Vo = oracle.sample_direct(img, c.dxy, rounded(c.u[idx], d), rounded(c.v[idx], d), c.PA,
                                  c.dRA, c.dDec, inc)
        ref[d] = (Vo, max(float(np.max(np.abs(Vo))), abs(float(np.sum(img)))))
        del img
    return kind, c, idx, ref


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_16384_sampled_against_oracle(case16k, dtype):
    dev = device()
    gal = _gal()
    kind, c, idx, ref = case16k
    Vo, scale = ref[dtype]
    print(f"16384 {kind} {np.dtype(dtype).name}", flush=True)
    u, v = t(c.u, dtype, dev), t(c.v, dtype, dev)
    if kind == "image":
        model = t(c.image, dtype, dev)
        Vg = gal.sampleImage(model, c.dxy, u, v, c.PA, c.dRA, c.dDec, c.inc)
    else:
        model = t(c.I, dtype, dev)
        Vg = gal.sampleProfile(model, c.Rmin, c.dR, N, c.dxy, u, v, c.inc, c.PA, c.dRA, c.dDec)
    Vg = Vg.cpu().numpy()[idx]
    err = float(np.max(np.abs(Vg - Vo)))
    assert err <= TOL_V[dtype] * scale, (err, scale)
    # chi^2 of a dataset holding the sampled points (observations: the
    # oracle's model plus noise) against the oracle's chi^2
    re = Vo.real + c.noise_re[idx]
    im = Vo.imag + c.noise_im[idx]
    w = c.w[idx]
    ds = gal.Dataset(*(t(a, dtype, dev) for a in (c.u[idx], c.v[idx], re, im, w)))
    if kind == "image":
        c2g = float(ds.chi2Image(model, c.dxy, c.PA, c.dRA, c.dDec, c.inc))
    else:
        c2g = float(ds.chi2Profile(model, c.Rmin, c.dR, N, c.dxy, c.inc, c.PA, c.dRA, c.dDec))
    ds.close()
    ro, io, wo = (rounded(a, dtype) for a in (re, im, w))
    c2o = oracle.chi2(Vo, ro, io, wo)
    dV = np.abs(Vg - Vo) + np.abs(Vo) * np.finfo(dtype).eps
    assert abs(c2g - c2o) <= chi2_bound(c2o, dV, wo), (c2g, c2o)


def test_16384_refused_where_unsupported():
    dev = device()
    gal = _gal()
    from paper_1709_06999_amd import GalarioError

    import ctypes

    import torch
    from paper_1709_06999_amd import _native

    # gradients keep the 8192 limit: refused on the host, before any launch
    c = wl.random_case(64, 100, seed=5, kind="profile")
    d = np.float64
    ds = gal.Dataset(*(t(a, d, dev) for a in (c.u, c.v, c.noise_re, c.noise_im, c.w)))
    I = t(c.I, d, dev)
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        ds.chi2Profile_grad(I, c.Rmin, c.dR, N, c.dxy / 256, c.inc, c.PA)
    ws = torch.zeros(1 << 20, dtype=torch.uint8, device=dev)
    out = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
    g = torch.empty_like(I)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    rc = _native.lib().gal_chi2Profile_grad_ds_d(ds._h, p(I), I.numel(), c.Rmin, c.dR, N,
                                                 c.dxy / 256, c.inc, c.PA, 0.0, 0.0, p(out), p(g),
                                                 p(ws), ws.numel(), None)
    assert rc == _native.GAL_ERR_SIZE
    torch.cuda.synchronize()
    assert float(out[0]) == -1.0
    ds.close()
    # 32768 is beyond every call
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        gal.sampleProfile(t(c.I, d, dev), c.Rmin, c.dR, 2 * N, c.dxy, t(c.u, d, dev),
                          t(c.v, d, dev))
