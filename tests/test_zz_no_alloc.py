"""The allocation-free chi2Profile entry point (gal_chi2Profile_ds_scratch_d)
against the same call with a caller's workspace (gal_chi2Profile_ds_d), both
through the C ABI.  Both run the same kernels with the same fixed-order
reduction, so the two chi^2 values must agree bit for bit, on consecutive
calls whose second input is smaller than the first."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from gpu_util import device, t

pytestmark = pytest.mark.gpu


def _p(x):
    return ctypes.c_void_p(x.data_ptr())


def _case(wl, dev):
    import paper_1709_06999_amd as gal

    # observed = noise only: chi^2 = sum w |noise - V|^2, a full-size sum either way
    ds = gal.Dataset(*(t(a, np.float64, dev) for a in (wl.u, wl.v, wl.noise_re, wl.noise_im,
                                                         wl.w)))
    return ds, t(wl.I, np.float64, dev)


def _both(L, ds, I, wl, dev):
    import torch

    ws_bytes = L.gal_workspace_bytes_d(wl.N, wl.M)
    ws = torch.zeros(ws_bytes, dtype=torch.uint8, device=dev)
    out = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
    args = (I.numel(), wl.Rmin, wl.dR, wl.N, wl.dxy, wl.inc, wl.PA, wl.dRA, wl.dDec)
    rc = L.gal_chi2Profile_ds_d(ds._h, _p(I), *args,
                                ctypes.c_void_p(out.data_ptr()), _p(ws), ws_bytes, None)
    assert rc == 0, L.gal_last_error()
    rc = L.gal_chi2Profile_ds_scratch_d(ds._h, _p(I), *args,
                                        ctypes.c_void_p(out.data_ptr() + 8), None)
    assert rc == 0, L.gal_last_error()
    torch.cuda.synchronize()
    a, b = out.cpu().numpy()
    return float(a), float(b)


def test_scratch_entry_matches_workspace_entry():
    dev = device()
    import torch

    import workloads as wl_mod
    from paper_1709_06999_amd import _native

    torch.cuda.set_device(dev)
    L = _native.lib()
    big = wl_mod.profile_2048(M=1_000_000)      # 2048^2, Nr = 4096, M = 1e6
    small = wl_mod.random_case(256, 20_000, seed=41, kind="profile")
    print(f"scratch entry: {big.name} then {small.name}", flush=True)
    ds_big, I_big = _case(big, dev)
    ds_small, I_small = _case(small, dev)
    a1, b1 = _both(L, ds_big, I_big, big, dev)
    assert np.isfinite(a1) and a1 > 0.0
    assert b1 == a1, (a1, b1)
    # second call, smaller image and fewer points: the scratch keeps the
    # first call's contents, which must not leak into this result
    a2, b2 = _both(L, ds_small, I_small, small, dev)
    assert np.isfinite(a2) and a2 > 0.0
    assert b2 == a2, (a2, b2)
    # and the larger one again
    a3, b3 = _both(L, ds_big, I_big, big, dev)
    assert a3 == a1 and b3 == a1
    # the Python binding calls the same entry point
    c = float(ds_small.chi2Profile_scratch(I_small, small.Rmin, small.dR, small.N, small.dxy,
                                           small.inc, small.PA, small.dRA, small.dDec))
    assert c == a2
    ds_big.close()
    ds_small.close()


def test_scratch_entry_refuses_sizes_beyond_the_scratch():
    dev = device()
    import torch

    import workloads as wl_mod
    from paper_1709_06999_amd import _native

    torch.cuda.set_device(dev)
    L = _native.lib()
    small = wl_mod.random_case(256, 1000, seed=42, kind="profile")
    ds, I = _case(small, dev)
    out = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    # 4096^2 needs 4097 x 2049 x 16 bytes of intermediate spectrum: above the scratch
    assert L.gal_workspace_bytes_d(4096, small.M) > _native.GAL_SCRATCH_BYTES
    rc = L.gal_chi2Profile_ds_scratch_d(ds._h, _p(I), I.numel(), small.Rmin,
                                        small.dR, 4096, small.dxy / 16, small.inc, small.PA,
                                        small.dRA, small.dDec, _p(out), None)
    assert rc == _native.GAL_ERR_WORKSPACE
    assert b"scratch" in L.gal_last_error()
    rc = L.gal_chi2Profile_ds_scratch_d(None, _p(I), I.numel(), small.Rmin, small.dR, 256,
                                        small.dxy, small.inc, small.PA, small.dRA, small.dDec,
                                        _p(out), None)
    assert rc == -1
    torch.cuda.synchronize()
    assert float(out.cpu()[0]) == -1.0   # nothing was enqueued
    ds.close()
