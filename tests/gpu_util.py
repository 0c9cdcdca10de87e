"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
from __future__ import annotations

import math

import numpy as np
import pytest

TOL_V = {np.float64: 1e-10, np.float32: 1e-4}


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def t(a, dtype, dev):
    import torch

    td = torch.float64 if dtype == np.float64 else torch.float32
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype), dtype=td, device=dev)


def rounded(a, dtype):
    """The array as the GPU sees it (FP32 rounding), promoted exactly to FP64."""
    return np.asarray(np.asarray(a, dtype=dtype), dtype=np.float64)


def assert_vis_close(Vg, Vo, dtype, what=""):
    Vg = np.asarray(Vg, dtype=np.complex128)
    scale = np.max(np.abs(Vo))
    err = np.max(np.abs(Vg - Vo)) if Vo.size else 0.0
    tol = TOL_V[dtype] * scale
    assert err <= tol, f"{what}: max|dV| = {err:.3e} > {tol:.3e} (max|V| = {scale:.3e})"
    return err / scale if scale > 0 else 0.0


def chi2_bound(c2_ref, dV, w):
    """|chi2' - chi2| allowed for model errors dV (Cauchy-Schwarz) plus a
    summation-order slack."""
    e = float(np.sum(w * np.abs(dV) ** 2))
    return 2.0 * math.sqrt(max(c2_ref, 0.0) * e) + e + 1e-12 * abs(c2_ref) + 1e-300
