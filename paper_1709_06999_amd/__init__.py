"""MI355X (gfx950) visibility / chi-square library after GALARIO
(Tazzari, Beaujean & Testi 2018, arXiv:1709.06999).

Thin torch binding of the C ABI in ``include/galario_hip.h``: it checks
tensors, picks the precision from their dtype (float64 -> ``_d``,
float32 -> ``_f``), passes device pointers and the current HIP stream, and
keeps one workspace per (device, dtype).  Every step of the path runs in the
library's HIP kernels; there is no other implementation behind these calls.

The calls follow the paper's Python interface (Sec. 2.2):

    sampleImage(image, dxy, u, v, PA=0, dRA=0, dDec=0, inc=0)  -> complex V [M]
    sampleProfile(I, Rmin, dR, Nxy, dxy, u, v, inc=0, PA=0, dRA=0, dDec=0)
    chi2Image(image, dxy, u, v, Re, Im, w, PA=0, dRA=0, dDec=0, inc=0) -> 0-d tensor
    chi2Profile(I, Rmin, dR, Nxy, dxy, u, v, Re, Im, w, inc=0, PA=0, dRA=0, dDec=0)
    sweep(I, Rmin, dR, Nxy, dxy, inc=0) -> image [Nxy, Nxy]

Angles in radians, uv in wavelengths.  chi2 results stay on the device as
0-d float64 tensors (call ``float()`` to synchronise).
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

from . import _native
from ._native import GalarioError, check

__all__ = [
    "sweep", "sampleImage", "sampleProfile", "chi2Image", "chi2Profile", "spectrum",
    "sample_spectrum", "Dataset", "Workspace", "read_status", "timing", "GalarioError",
    "version", "init", "autotune", "autotune_batch", "tune_get", "tune_set", "Batch", "profile_batch",
    "JOB_IMAGE", "JOB_PROFILE", "batch_exec", "chi2Image_grad", "chi2Profile_grad", "chi2_profile", "chi2_image",
    "get_image_size", "STATUS_UV", "STATUS_GEO", "batch_exec_status", "exec_workspace_bytes",
]

JOB_IMAGE = 0
JOB_PROFILE = 1


def _lib():
    return _native.lib()


def version() -> str:
    return _lib().gal_version().decode()


def init(device: int | None = None):
    dev = torch.cuda.current_device() if device is None else int(device)
    check(_lib().gal_init(dev), "gal_init")


def _sfx(dtype: torch.dtype) -> str:
    if dtype == torch.float64:
        return "_d"
    if dtype == torch.float32:
        return "_f"
    raise TypeError(f"arrays must be float64 or float32, got {dtype}")


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _arr(t, name: str, dtype: torch.dtype, device: torch.device, n: int | None = None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t


def _device_of(t: torch.Tensor) -> torch.device:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("inputs must be torch tensors on a GPU (device 'cuda')")
    return t.device


class Workspace:
    """Device scratch memory for the library calls on one device and dtype.

    Grows on demand; its 256-byte control block is zero at allocation.  Calls
    that share a workspace must run on one stream (they do when they use the
    default per-device workspace from the current stream)."""

    def __init__(self, device: torch.device, dtype: torch.dtype):
        self.device = torch.device(device)
        self.dtype = dtype
        self.buf = torch.zeros(0, dtype=torch.uint8, device=self.device)

    def reserve(self, Nxy: int, M: int, grad_Nr: int | None = None) -> torch.Tensor:
        """Grow to the bytes a call needs (grad_Nr: a gradient call, with the
        profile length or 0 for images)."""
        if grad_Nr is None:
            need = getattr(_lib(), "gal_workspace_bytes" + _sfx(self.dtype))(int(Nxy), int(M))
        else:
            need = getattr(_lib(), "gal_grad_workspace_bytes" + _sfx(self.dtype))(
                int(Nxy), int(M), int(grad_Nr))
        if need == 0:
            raise GalarioError(-2, f"workspace size (Nxy={Nxy}, M={M})")
        return self.reserve_bytes(need)

    def reserve_bytes(self, need: int) -> torch.Tensor:
        if self.buf.numel() < need:
            self.buf = torch.zeros(int(need), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws: dict = {}


def _ws(device: torch.device, dtype: torch.dtype, ws: Workspace | None) -> Workspace:
    if ws is not None:
        return ws
    key = (device.index if device.index is not None else torch.cuda.current_device(), dtype)
    if key not in _default_ws:
        _default_ws[key] = Workspace(torch.device("cuda", key[0]), dtype)
    return _default_ws[key]


STATUS_UV = 1    # a uv point fell outside the half spectrum (its samples are NaN)
STATUS_GEO = 2   # a batch job's geometry row failed its checks (its chi^2 is NaN)


def _read_status_buf(buf: torch.Tensor, dev: torch.device) -> int:
    st = ctypes.c_int(0)
    with torch.cuda.device(dev):
        check(_lib().gal_read_status(_ptr(buf), _stream(dev), ctypes.byref(st)), "gal_read_status")
    return int(st.value)


def read_status(dtype: torch.dtype = torch.float64, device=None, ws: Workspace | None = None) -> int:
    """Status bits of the calls on this workspace since the last read, then
    cleared: STATUS_UV if a uv point of a raw-array call fell outside the half
    spectrum (its samples are NaN), else 0.  Synchronises the stream."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    w = _ws(dev, dtype, ws)
    if w.buf.numel() == 0:
        return 0
    return _read_status_buf(w.buf, dev)


# ----------------------------------------------------------------------------
def sweep(I, Rmin, dR, Nxy, dxy, inc=0.0):
    dev = _device_of(I)
    _arr(I, "I", I.dtype, dev)
    out = torch.empty((int(Nxy), int(Nxy)), dtype=I.dtype, device=dev)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_sweep" + _sfx(I.dtype))(
            _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy), float(inc),
            _ptr(out), _stream(dev)), "sweep")
    return out


def sampleImage(image, dxy, u, v, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0, ws: Workspace | None = None):
    dev = _device_of(image)
    dt = image.dtype
    N = image.shape[0]
    if image.dim() != 2 or image.shape[1] != N:
        raise ValueError("image must be square [Nxy, Nxy]")
    _arr(image, "image", dt, dev)
    M = u.numel()
    _arr(u, "u", dt, dev, M), _arr(v, "v", dt, dev, M)
    out = torch.empty((M, 2), dtype=dt, device=dev)
    w = _ws(dev, dt, ws).reserve(N, M)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_sampleImage" + _sfx(dt))(
            _ptr(image), N, float(dxy), _ptr(u), _ptr(v), M, float(PA), float(dRA), float(dDec),
            float(inc), _ptr(out), _ptr(w), w.numel(), _stream(dev)), "sampleImage")
    return torch.view_as_complex(out)


def sampleProfile(I, Rmin, dR, Nxy, dxy, u, v, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                  ws: Workspace | None = None):
    dev = _device_of(I)
    dt = I.dtype
    _arr(I, "I", dt, dev)
    M = u.numel()
    _arr(u, "u", dt, dev, M), _arr(v, "v", dt, dev, M)
    out = torch.empty((M, 2), dtype=dt, device=dev)
    w = _ws(dev, dt, ws).reserve(Nxy, M)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_sampleProfile" + _sfx(dt))(
            _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy), _ptr(u), _ptr(v), M,
            float(inc), float(PA), float(dRA), float(dDec), _ptr(out), _ptr(w), w.numel(),
            _stream(dev)), "sampleProfile")
    return torch.view_as_complex(out)


def chi2Image(image, dxy, u, v, re, im, w, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
              ws: Workspace | None = None, out: torch.Tensor | None = None):
    dev = _device_of(image)
    dt = image.dtype
    N = image.shape[0]
    if image.dim() != 2 or image.shape[1] != N:
        raise ValueError("image must be square [Nxy, Nxy]")
    _arr(image, "image", dt, dev)
    M = u.numel()
    for t, n in ((u, "u"), (v, "v"), (re, "Re"), (im, "Im"), (w, "w")):
        _arr(t, n, dt, dev, M)
    res = torch.empty((), dtype=torch.float64, device=dev) if out is None else out
    wsb = _ws(dev, dt, ws).reserve(N, M)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_chi2Image" + _sfx(dt))(
            _ptr(image), N, float(dxy), _ptr(u), _ptr(v), _ptr(re), _ptr(im), _ptr(w), M,
            float(PA), float(dRA), float(dDec), float(inc), _ptr(res), _ptr(wsb), wsb.numel(),
            _stream(dev)), "chi2Image")
    return res


def chi2Profile(I, Rmin, dR, Nxy, dxy, u, v, re, im, w, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                ws: Workspace | None = None, out: torch.Tensor | None = None):
    dev = _device_of(I)
    dt = I.dtype
    _arr(I, "I", dt, dev)
    M = u.numel()
    for t, n in ((u, "u"), (v, "v"), (re, "Re"), (im, "Im"), (w, "w")):
        _arr(t, n, dt, dev, M)
    res = torch.empty((), dtype=torch.float64, device=dev) if out is None else out
    wsb = _ws(dev, dt, ws).reserve(Nxy, M)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_chi2Profile" + _sfx(dt))(
            _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy), _ptr(u), _ptr(v),
            _ptr(re), _ptr(im), _ptr(w), M, float(inc), float(PA), float(dRA), float(dDec),
            _ptr(res), _ptr(wsb), wsb.numel(), _stream(dev)), "chi2Profile")
    return res


def chi2Image_grad(image, dxy, u, v, re, im, w, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
                   ws: Workspace | None = None):
    """(chi^2 as a 0-d device tensor, d chi^2 / d image [Nxy, Nxy])."""
    dev = _device_of(image)
    dt = image.dtype
    N = image.shape[0]
    _arr(image, "image", dt, dev, N * N)
    M = u.numel()
    for t_, n in ((u, "u"), (v, "v"), (re, "Re"), (im, "Im"), (w, "w")):
        _arr(t_, n, dt, dev, M)
    c2 = torch.empty((), dtype=torch.float64, device=dev)
    g = torch.empty_like(image)
    wsb = _ws(dev, dt, ws).reserve(N, M, 0)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_chi2Image_grad" + _sfx(dt))(
            _ptr(image), N, float(dxy), _ptr(u), _ptr(v), _ptr(re), _ptr(im), _ptr(w), M,
            float(PA), float(dRA), float(dDec), float(inc), _ptr(c2), _ptr(g), _ptr(wsb),
            wsb.numel(), _stream(dev)), "chi2Image_grad")
    return c2, g


def chi2Profile_grad(I, Rmin, dR, Nxy, dxy, u, v, re, im, w, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                     ws: Workspace | None = None):
    """(chi^2 as a 0-d device tensor, d chi^2 / d I [Nr])."""
    dev = _device_of(I)
    dt = I.dtype
    _arr(I, "I", dt, dev)
    M = u.numel()
    for t_, n in ((u, "u"), (v, "v"), (re, "Re"), (im, "Im"), (w, "w")):
        _arr(t_, n, dt, dev, M)
    c2 = torch.empty((), dtype=torch.float64, device=dev)
    g = torch.empty_like(I)
    wsb = _ws(dev, dt, ws).reserve(Nxy, M, I.numel())
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_chi2Profile_grad" + _sfx(dt))(
            _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy), _ptr(u), _ptr(v),
            _ptr(re), _ptr(im), _ptr(w), M, float(inc), float(PA), float(dRA), float(dDec),
            _ptr(c2), _ptr(g), _ptr(wsb), wsb.numel(), _stream(dev)), "chi2Profile_grad")
    return c2, g


def spectrum(image, ws: Workspace | None = None):
    """Half spectrum G [Nxy, Nxy/2+1] (complex) of the image with its origin at
    pixel (Nxy/2, Nxy/2); row p is frequency p - Nxy [p >= Nxy/2]."""
    dev = _device_of(image)
    dt = image.dtype
    N = image.shape[0]
    _arr(image, "image", dt, dev, N * N)
    out = torch.empty((N, N // 2 + 1, 2), dtype=dt, device=dev)
    wsb = _ws(dev, dt, ws).reserve(N, 0)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_spectrum" + _sfx(dt))(
            _ptr(image), N, _ptr(out), _ptr(wsb), wsb.numel(), _stream(dev)), "spectrum")
    return torch.view_as_complex(out)


def sample_spectrum(spec, dxy, u, v, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
                    ws: Workspace | None = None):
    """Sample a half spectrum laid out as ``spectrum`` returns it."""
    dev = _device_of(spec)
    if not spec.is_complex():
        raise TypeError("spec must be complex")
    sr = torch.view_as_real(spec)
    dt = sr.dtype
    N = spec.shape[0]
    if spec.shape != (N, N // 2 + 1) or not spec.is_contiguous():
        raise ValueError("spec must be a contiguous [Nxy, Nxy/2+1] complex tensor")
    M = u.numel()
    _arr(u, "u", dt, dev, M), _arr(v, "v", dt, dev, M)
    out = torch.empty((M, 2), dtype=dt, device=dev)
    wsb = _ws(dev, dt, ws).reserve(N, M)
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_sample_spectrum" + _sfx(dt))(
            _ptr(sr), N, float(dxy), _ptr(u), _ptr(v), M, float(PA), float(dRA), float(dDec),
            float(inc), _ptr(out), _ptr(wsb), wsb.numel(), _stream(dev)), "sample_spectrum")
    return torch.view_as_complex(out)


# ----------------------------------------------------------------------------
def get_image_size(u, v, PB: float = 0.0, f_min: float = 5.0, f_max: float = 2.5,
                   Gamma: float = 0.6, smooth: bool = False):
    """(Nxy, dxy [rad]) for the uv points by the criteria of Sec. 3.4
    (gal_image_size): the image spans f_min times the largest recoverable scale
    Gamma / rho_min (or, with PB > 0, the primary beam of FWHM PB [rad]), the
    grid reaches f_max times the longest baseline, Nxy a power of two (smooth:
    the smallest even 2^a 3^b 5^c, gal_image_size_smooth).  u, v: numpy arrays
    or tensors (read on the host)."""
    import numpy as np

    host = [np.ascontiguousarray(x.detach().cpu().numpy() if isinstance(x, torch.Tensor) else x)
            for x in (u, v)]
    if host[0].dtype != host[1].dtype or host[0].dtype not in (np.float64, np.float32):
        raise TypeError("u and v must both be float64 or both float32")
    if host[0].shape != host[1].shape:
        raise ValueError("u and v must have the same shape")
    sfx = "_d" if host[0].dtype == np.float64 else "_f"
    lo, hi = ctypes.c_double(0), ctypes.c_double(0)
    check(getattr(_lib(), "gal_uv_range" + sfx)(host[0].ctypes.data, host[1].ctypes.data,
                                                host[0].size, ctypes.byref(lo), ctypes.byref(hi)),
          "get_image_size")
    n, d = ctypes.c_int(0), ctypes.c_double(0)
    fn = _lib().gal_image_size_smooth if smooth else _lib().gal_image_size
    check(fn(lo.value, hi.value, float(f_min), float(f_max), float(PB), float(Gamma),
             ctypes.byref(n), ctypes.byref(d)), "get_image_size")
    return int(n.value), float(d.value)


class Dataset:
    """An observation registered once in library-owned device memory.

    Calls on a dataset check the uv range on the host and transform only the
    part of the half spectrum its points reach (same samples as the full
    spectrum)."""

    def __init__(self, u, v, re=None, im=None, w=None):
        dev = _device_of(u)
        dt = u.dtype
        M = u.numel()
        _arr(u, "u", dt, dev, M), _arr(v, "v", dt, dev, M)
        if re is not None or im is not None or w is not None:
            for t, n in ((re, "Re"), (im, "Im"), (w, "w")):
                _arr(t, n, dt, dev, M)
        self.device, self.dtype, self.M = dev, dt, M
        self.has_obs = re is not None
        h = ctypes.c_void_p(0)
        with torch.cuda.device(dev):
            check(getattr(_lib(), "gal_dataset_create" + _sfx(dt))(
                _ptr(u), _ptr(v), _ptr(re), _ptr(im), _ptr(w), M, _stream(dev), ctypes.byref(h)),
                "Dataset")
        self._h = h
        m, rho, prec = ctypes.c_int64(0), ctypes.c_double(0), ctypes.c_int(0)
        check(_lib().gal_dataset_info(h, ctypes.byref(m), ctypes.byref(rho), ctypes.byref(prec)),
              "gal_dataset_info")
        self.rho_max = float(rho.value)

    def image_size(self, PB: float = 0.0, f_min: float = 5.0, f_max: float = 2.5,
                   Gamma: float = 0.6, smooth: bool = False):
        """(Nxy, dxy) for this dataset's uv range (as ``get_image_size``)."""
        n, d = ctypes.c_int(0), ctypes.c_double(0)
        fn = _lib().gal_dataset_image_size_smooth if smooth else _lib().gal_dataset_image_size
        check(fn(self._h, float(f_min), float(f_max), float(PB), float(Gamma), ctypes.byref(n),
                 ctypes.byref(d)), "Dataset.image_size")
        return int(n.value), float(d.value)

    def geometry(self, Nxy, dxy):
        """(Q, P): columns [0, Q) and rows [-P, P] of the half spectrum that
        calls on this dataset transform for an Nxy image of pixel dxy."""
        q, p = ctypes.c_int(0), ctypes.c_int(0)
        check(_lib().gal_dataset_geometry(self._h, int(Nxy), float(dxy), ctypes.byref(q),
                                          ctypes.byref(p)), "gal_dataset_geometry")
        return int(q.value), int(p.value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            with torch.cuda.device(self.device):
                _lib().gal_dataset_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, t, name):
        return _arr(t, name, self.dtype, self.device)

    def chi2Image(self, image, dxy, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
                  ws: Workspace | None = None, out: torch.Tensor | None = None):
        self._chk(image, "image")
        N = image.shape[0]
        res = torch.empty((), dtype=torch.float64, device=self.device) if out is None else out
        wsb = _ws(self.device, self.dtype, ws).reserve(N, self.M)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_chi2Image_ds" + _sfx(self.dtype))(
                self._h, _ptr(image), N, float(dxy), float(PA), float(dRA), float(dDec), float(inc),
                _ptr(res), _ptr(wsb), wsb.numel(), _stream(self.device)), "Dataset.chi2Image")
        return res

    def chi2Profile(self, I, Rmin, dR, Nxy, dxy, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                    ws: Workspace | None = None, out: torch.Tensor | None = None):
        self._chk(I, "I")
        res = torch.empty((), dtype=torch.float64, device=self.device) if out is None else out
        wsb = _ws(self.device, self.dtype, ws).reserve(Nxy, self.M)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_chi2Profile_ds" + _sfx(self.dtype))(
                self._h, _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy),
                float(inc), float(PA), float(dRA), float(dDec), _ptr(res), _ptr(wsb), wsb.numel(),
                _stream(self.device)), "Dataset.chi2Profile")
        return res

    def chi2Profile_scratch(self, I, Rmin, dR, Nxy, dxy, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                            out: torch.Tensor | None = None):
        """chi2Profile with the library's static scratch workspace (FP64 datasets
        only): the C call allocates nothing, for callers that cannot allocate
        (pass `out` to allocate nothing here either).  Calls on one device share
        the scratch, so calls on different streams must not overlap."""
        if self.dtype != torch.float64:
            raise TypeError("chi2Profile_scratch needs an FP64 dataset")
        self._chk(I, "I")
        res = torch.empty((), dtype=torch.float64, device=self.device) if out is None else out
        with torch.cuda.device(self.device):
            check(_lib().gal_chi2Profile_ds_scratch_d(
                self._h, _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy),
                float(inc), float(PA), float(dRA), float(dDec), _ptr(res), _stream(self.device)),
                "Dataset.chi2Profile_scratch")
        return res

    def chi2Image_grad(self, image, dxy, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
                       ws: Workspace | None = None):
        """(chi^2 0-d tensor, d chi^2 / d image)."""
        self._chk(image, "image")
        N = image.shape[0]
        c2 = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty_like(image)
        wsb = _ws(self.device, self.dtype, ws).reserve(N, self.M, 0)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_chi2Image_grad_ds" + _sfx(self.dtype))(
                self._h, _ptr(image), N, float(dxy), float(PA), float(dRA), float(dDec), float(inc),
                _ptr(c2), _ptr(g), _ptr(wsb), wsb.numel(), _stream(self.device)),
                "Dataset.chi2Image_grad")
        return c2, g

    def chi2Profile_grad(self, I, Rmin, dR, Nxy, dxy, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                         ws: Workspace | None = None):
        """(chi^2 0-d tensor, d chi^2 / d I)."""
        self._chk(I, "I")
        c2 = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty_like(I)
        wsb = _ws(self.device, self.dtype, ws).reserve(Nxy, self.M, I.numel())
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_chi2Profile_grad_ds" + _sfx(self.dtype))(
                self._h, _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy),
                float(inc), float(PA), float(dRA), float(dDec), _ptr(c2), _ptr(g), _ptr(wsb),
                wsb.numel(), _stream(self.device)), "Dataset.chi2Profile_grad")
        return c2, g

    def _geo_ws(self, Nxy, ws):
        need = getattr(_lib(), "gal_geograd_workspace_bytes" + _sfx(self.dtype))(int(Nxy), self.M)
        if need == 0:
            raise GalarioError(-2, f"geograd workspace size (Nxy={Nxy})")
        return _ws(self.device, self.dtype, ws).reserve_bytes(int(need))

    def chi2Image_geograd(self, image, dxy, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
                          ws: Workspace | None = None):
        """(chi^2 0-d tensor, d chi^2 / d [PA, dRA, dDec, inc] as a float64 tensor [4])."""
        self._chk(image, "image")
        N = image.shape[0]
        c2 = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(4, dtype=torch.float64, device=self.device)
        wsb = self._geo_ws(N, ws)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_chi2Image_geograd_ds" + _sfx(self.dtype))(
                self._h, _ptr(image), N, float(dxy), float(PA), float(dRA), float(dDec),
                float(inc), _ptr(c2), _ptr(g), _ptr(wsb), wsb.numel(), _stream(self.device)),
                "Dataset.chi2Image_geograd")
        return c2, g

    def chi2Profile_geograd(self, I, Rmin, dR, Nxy, dxy, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                            ws: Workspace | None = None):
        """(chi^2 0-d tensor, d chi^2 / d [PA, dRA, dDec, inc] as a float64 tensor [4]);
        the inclination derivative goes through the swept image."""
        self._chk(I, "I")
        c2 = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(4, dtype=torch.float64, device=self.device)
        wsb = self._geo_ws(Nxy, ws)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_chi2Profile_geograd_ds" + _sfx(self.dtype))(
                self._h, _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy),
                float(inc), float(PA), float(dRA), float(dDec), _ptr(c2), _ptr(g), _ptr(wsb),
                wsb.numel(), _stream(self.device)), "Dataset.chi2Profile_geograd")
        return c2, g

    def _scene_jobs(self, sources):
        """Jobs of one scene from source dicts: kind ("image" / "profile" or
        JOB_*), model (image [Nxy, Nxy] or profile [Nr]; None with share),
        dxy, Nxy (profiles, and sharing images), Rmin, dR (profiles), inc,
        PA, dRA, dDec (default 0), share (index of the source whose spectrum
        this one reads)."""
        if not sources:
            raise ValueError("a scene needs at least one source")
        jobs = []
        for k, s in enumerate(sources):
            kind = s["kind"]
            kind = {"image": JOB_IMAGE, "profile": JOB_PROFILE}.get(kind, kind)
            if kind not in (JOB_IMAGE, JOB_PROFILE):
                raise ValueError(f"source {k}: kind must be 'image' or 'profile'")
            m = s.get("model")
            if kind == JOB_IMAGE and m is not None:
                N = m.shape[0]
            else:
                N = s.get("Nxy")
                if N is None and s.get("share") is not None:
                    N = sources[s["share"]].get("Nxy") or sources[s["share"]]["model"].shape[0]
            geo = torch.tensor([float(s.get(key, 0.0)) for key in
                                ("Rmin", "dR", "inc", "PA", "dRA", "dDec")],
                               dtype=torch.float64, device=self.device)
            jobs.append({"ds": self, "kind": kind, "Nxy": int(N), "dxy": float(s["dxy"]),
                         "model": m, "geo": geo, "scene": 1, "share": s.get("share")})
        return jobs

    def sampleSources(self, sources, ws: Workspace | None = None):
        """Model visibilities (complex [M]) of a field of several sources:
        the sum of each source's visibilities, each placed and oriented by its
        own geometry (one sampling pass; sources that share a spectrum are
        transformed once)."""
        jobs = self._scene_jobs(sources)
        vis = torch.empty(self.M, dtype=_COMPLEX[self.dtype], device=self.device)
        jobs[0]["vis"] = vis
        batch_exec(jobs, ws=ws)
        return vis

    def chi2Sources(self, sources, grad: bool = False, ws: Workspace | None = None):
        """chi^2 (0-d tensor) of the field of several sources against the
        observations; with grad=True also a list with d chi^2 / d model of
        every source that owns a model (None for sources that share one: their
        part is in the owner's)."""
        jobs = self._scene_jobs(sources)
        grads = None
        if grad:
            grads = [torch.empty_like(j["model"]) if j["model"] is not None else None
                     for j in jobs]
        c2 = batch_exec(jobs, grads, ws=ws)[0]
        return (c2, grads) if grad else c2

    def sampleImage(self, image, dxy, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0,
                    ws: Workspace | None = None):
        self._chk(image, "image")
        N = image.shape[0]
        out = torch.empty((self.M, 2), dtype=self.dtype, device=self.device)
        wsb = _ws(self.device, self.dtype, ws).reserve(N, self.M)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_sampleImage_ds" + _sfx(self.dtype))(
                self._h, _ptr(image), N, float(dxy), float(PA), float(dRA), float(dDec), float(inc),
                _ptr(out), _ptr(wsb), wsb.numel(), _stream(self.device)), "Dataset.sampleImage")
        return torch.view_as_complex(out)

    def sampleProfile(self, I, Rmin, dR, Nxy, dxy, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0,
                      ws: Workspace | None = None):
        self._chk(I, "I")
        out = torch.empty((self.M, 2), dtype=self.dtype, device=self.device)
        wsb = _ws(self.device, self.dtype, ws).reserve(Nxy, self.M)
        with torch.cuda.device(self.device):
            check(getattr(_lib(), "gal_sampleProfile_ds" + _sfx(self.dtype))(
                self._h, _ptr(I), I.numel(), float(Rmin), float(dR), int(Nxy), float(dxy),
                float(inc), float(PA), float(dRA), float(dDec), _ptr(out), _ptr(wsb), wsb.numel(),
                _stream(self.device)), "Dataset.sampleProfile")
        return torch.view_as_complex(out)


# ----------------------------------------------------------------------------
_COMPLEX = {torch.float64: torch.complex128, torch.float32: torch.complex64}


def _job_array(jobs, dev: torch.device):
    """gal_job array of job dicts: ds, kind, Nxy, dxy, model, geo and the
    optional scene (int, 0 = alone), share (index of the job whose spectrum
    this one reads, or None) and vis (complex tensor [M] for the scene's
    visibilities)."""
    arr = (_native.GalJob * len(jobs))()
    for i, j in enumerate(jobs):
        ds = j["ds"]
        if ds.device != dev:
            raise ValueError(f"job {i}: dataset on {ds.device}, expected {dev}")
        m, geo = j.get("model"), j["geo"]
        share = j.get("share")
        share = 0 if share is None else int(share) + 1
        if m is None and not share:
            raise ValueError(f"job {i}: a model is needed unless the job shares a spectrum")
        if m is not None:
            _arr(m, "model", ds.dtype, dev)
        _arr(geo, "geo", torch.float64, dev, 6)
        vis = j.get("vis")
        if vis is not None:
            _arr(vis, "vis", _COMPLEX[ds.dtype], dev, ds.M)
        nr = int(m.numel()) if (m is not None and j["kind"] == JOB_PROFILE) else 0
        arr[i] = _native.GalJob(ds._h.value, int(j["kind"]), int(j["Nxy"]), float(j["dxy"]), nr,
                                m.data_ptr() if m is not None else None, geo.data_ptr(),
                                int(j.get("scene", 0)), share,
                                vis.data_ptr() if vis is not None else None)
    return arr


class Batch:
    """A planned list of chi^2 jobs evaluated together (gal_batch_*).

    ``jobs`` is a list of dicts with keys: ds (Dataset), kind (JOB_IMAGE or
    JOB_PROFILE), Nxy, dxy, model (device tensor: image [Nxy, Nxy] or
    profile [Nr]) and geo (device float64 tensor of 6 values: Rmin, dR, inc,
    PA, dRA, dDec), and optionally scene, share and vis: jobs with the same
    nonzero scene are the sources of one field, whose visibilities add up
    (their chi^2 entries are the scene's); share = k makes a job read the
    spectrum of job k of its scene (model may then be None); vis (complex
    tensor [M]) receives the scene's model visibilities.  The kernels read
    model and geo at every ``chi2()`` call, so update those tensors in place
    between calls; the plan (and any HIP graph captured around ``chi2``)
    stays valid as long as they live."""

    def __init__(self, jobs):
        if not jobs:
            raise ValueError("a batch needs at least one job")
        self.jobs = list(jobs)
        dev = self.jobs[0]["ds"].device
        arr = _job_array(self.jobs, dev)
        self.device = dev
        h = ctypes.c_void_p(0)
        with torch.cuda.device(dev):
            check(_lib().gal_batch_create(arr, len(self.jobs), ctypes.byref(h)), "Batch")
        self._h = h
        need = _lib().gal_batch_workspace_bytes(h)
        self.ws = torch.zeros(int(need), dtype=torch.uint8, device=dev)
        self.out = torch.empty(len(self.jobs), dtype=torch.float64, device=dev)

    def info(self):
        n, f, g = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        check(_lib().gal_batch_info(self._h, ctypes.byref(n), ctypes.byref(f), ctypes.byref(g)),
              "gal_batch_info")
        return {"jobs": n.value, "fft_groups": f.value, "sample_groups": g.value}

    def chi2(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """chi^2 of every job (device float64 tensor [n]), on the current stream."""
        res = self.out if out is None else out
        with torch.cuda.device(self.device):
            check(_lib().gal_batch_chi2(self._h, _ptr(res), _ptr(self.ws), self.ws.numel(),
                                        _stream(self.device)), "Batch.chi2")
        return res

    def status(self) -> int:
        """Status bits of the executions since the last read, then cleared
        (synchronises the current stream): STATUS_GEO if a job's geometry row
        failed its checks (that job's chi^2 is NaN)."""
        return _read_status_buf(self.ws, self.device)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            with torch.cuda.device(self.device):
                _lib().gal_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_batch(ds: "Dataset", I: torch.Tensor, geo: torch.Tensor, Nxy: int, dxy: float) -> Batch:
    """K profile jobs on one dataset: I [K, Nr] (dataset dtype), geo [K, 6]
    float64 rows {Rmin, dR, inc, PA, dRA, dDec}; both updated in place by the
    caller between evaluations."""
    if I.dim() != 2 or geo.shape != (I.shape[0], 6):
        raise ValueError("I must be [K, Nr] and geo [K, 6]")
    return Batch([{"ds": ds, "kind": JOB_PROFILE, "Nxy": Nxy, "dxy": dxy, "model": I[k],
                   "geo": geo[k]} for k in range(I.shape[0])])


_exec_ws: dict = {}


def batch_exec(jobs, grads=None, out: torch.Tensor | None = None,
               ws: Workspace | None = None) -> torch.Tensor:
    """One-shot chi^2 (and optional gradients) of a job list, planned at this
    call (gal_batch_exec): any mix of kinds, sizes, datasets and precisions.

    ``jobs`` as for ``Batch``; ``grads`` (optional) is a list with one entry
    per job: None (chi^2 only) or a device tensor of the model's shape and
    dtype that receives d chi^2 / d model (of the job's scene).  Returns chi^2 as a device float64
    tensor [n], on the current stream.  Nothing is allocated beyond the
    (growing, per-device) workspace."""
    jobs = list(jobs)
    if not jobs:
        raise ValueError("batch_exec needs at least one job")
    dev = jobs[0]["ds"].device
    arr = _job_array(jobs, dev)
    gp = None
    if grads is not None:
        if len(grads) != len(jobs):
            raise ValueError("grads needs one entry per job")
        gp = (ctypes.c_void_p * len(jobs))()
        for i, (j, g) in enumerate(zip(jobs, grads)):
            if g is not None:
                if j.get("model") is None:
                    raise ValueError(f"job {i}: a job without a model has no gradient output")
                _arr(g, "grad", j["ds"].dtype, dev, j["model"].numel())
                gp[i] = g.data_ptr()
    need = _lib().gal_batch_exec_workspace_bytes(arr, len(jobs), gp)
    if need == 0:  # the plan failed; gal_last_error says why
        raise GalarioError(_native.GAL_ERR_SIZE, "batch_exec plan")
    if ws is None:
        key = dev.index if dev.index is not None else torch.cuda.current_device()
        ws = _exec_ws.setdefault(key, Workspace(torch.device("cuda", key), torch.float64))
    buf = ws.reserve_bytes(int(need))
    res = torch.empty(len(jobs), dtype=torch.float64, device=dev) if out is None else out
    _arr(res, "out", torch.float64, dev, len(jobs))
    with torch.cuda.device(dev):
        check(_lib().gal_batch_exec(arr, len(jobs), _ptr(res), gp, _ptr(buf), buf.numel(),
                                    _stream(dev)), "batch_exec")
    return res


def batch_exec_status(device=None, ws: Workspace | None = None) -> int:
    """Status bits of the batch_exec calls on this workspace (the default one
    of the device if None) since the last read, then cleared."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    if ws is None:
        key = dev.index if dev.index is not None else torch.cuda.current_device()
        ws = _exec_ws.get(key)
    if ws is None or ws.buf.numel() == 0:
        return 0
    return _read_status_buf(ws.buf, dev)


def exec_workspace_bytes(specs) -> int:
    """Workspace bytes batch_exec needs for a job list, from the library's
    planner on the host (no device work).  ``specs`` holds one tuple per job:
    (dataset, kind, Nxy, dxy, Nr, grad) with Nr the profile length (0 for
    images) and grad whether the job has a gradient output."""
    n = len(specs)
    arr = (_native.GalJob * n)()
    gp = (ctypes.c_void_p * n)()
    any_grad = False
    for i, (ds, kind, Nxy, dxy, Nr, grad) in enumerate(specs):
        # the planner reads no model or geometry value: any non-NULL address
        arr[i] = _native.GalJob(ds._h.value, int(kind), int(Nxy), float(dxy), int(Nr), 256, 256,
                                0, 0, None)
        gp[i] = 256 if grad else None
        any_grad = any_grad or bool(grad)
    need = _lib().gal_batch_exec_workspace_bytes(arr, n, gp if any_grad else None)
    if need == 0:
        raise GalarioError(_native.GAL_ERR_SIZE, "exec_workspace_bytes")
    return int(need)


# ----------------------------------------------------------------------------
# FFT schedule autotuning
def autotune(Nxy: int, dtype=torch.float64, frac: float = 1.0, device=None, times=None) -> list:
    """Time every FFT variant for this image size on the device and keep the
    fastest (see gal_autotune_*); returns the chosen variant per pass
    [rows_image, cols, rows_sym, cols_sym].  With GALARIO_HIP_TUNE_CACHE set
    to a JSON file path the choice is also stored there.  ``times``, if a
    dict, receives the per-variant launch times in ms."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    chosen = (ctypes.c_int * 4)()
    tms = (ctypes.c_double * 12)()
    with torch.cuda.device(dev):
        check(getattr(_lib(), "gal_autotune" + _sfx(dtype))(int(Nxy), float(frac), _stream(dev),
                                                             chosen, tms), "autotune")
    if isinstance(times, dict):
        names = ["rows_image", "cols", "rows_sym", "cols_sym"]
        for k in range(4):
            times[names[k]] = [round(tms[3 * k + v], 5) for v in range(3)]
    res = [int(c) for c in chosen]
    path = os.environ.get("GALARIO_HIP_TUNE_CACHE")
    if path:
        cache = _read_cache(path)
        cache[f"{8 if dtype == torch.float64 else 4}:{int(Nxy)}"] = res
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return res


def autotune_batch(batch: "Batch", Nxy: int, dtype=torch.float64, reps: int = 10,
                   times=None) -> list:
    """Tune the FFT variants for a planned batch as it runs: time
    ``batch.chi2()`` under each variant of each pass the batch uses (one pass
    at a time, the others at their current choice) and keep the fastest.
    Call it before capturing the batch into a graph (a graph keeps the
    kernels it recorded).  ``times``, if a dict, receives ms per execution."""
    kinds = sorted({2 if j["kind"] == JOB_PROFILE else 0 for j in batch.jobs
                    if int(j["Nxy"]) == int(Nxy) and j["ds"].dtype == dtype})
    best = tune_get(Nxy, dtype)
    names = ["rows_image", "cols", "rows_sym", "cols_sym"]
    dev = batch.device
    for k0 in kinds:
        for kind in (k0, k0 + 1):
            ms = []
            for var in range(3):
                trial = list(best)
                trial[kind] = var
                tune_set(Nxy, trial, dtype)
                batch.chi2()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                with torch.cuda.device(dev):
                    e0.record()
                    for _ in range(reps):
                        batch.chi2()
                    e1.record()
                e1.synchronize()
                ms.append(e0.elapsed_time(e1) / reps)
            best[kind] = int(min(range(3), key=lambda v: ms[v]))
            if isinstance(times, dict):
                times[names[kind]] = [round(x, 5) for x in ms]
    tune_set(Nxy, best, dtype)
    return best


def tune_get(Nxy: int, dtype=torch.float64) -> list:
    out = (ctypes.c_int * 4)()
    check(_lib().gal_tune_get(8 if dtype == torch.float64 else 4, int(Nxy), out), "tune_get")
    return [int(c) for c in out]


def tune_set(Nxy: int, chosen, dtype=torch.float64):
    arr = (ctypes.c_int * 4)(*[int(c) for c in chosen])
    check(_lib().gal_tune_set(8 if dtype == torch.float64 else 4, int(Nxy), arr), "tune_set")


def _read_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _load_tune_cache():
    path = os.environ.get("GALARIO_HIP_TUNE_CACHE")
    if not path:
        return
    for key, chosen in _read_cache(path).items():
        prec, n = key.split(":")
        check(_lib().gal_tune_set(int(prec), int(n), (ctypes.c_int * 4)(*chosen)), "tune cache")


# ----------------------------------------------------------------------------
class timing:
    """Per-kernel HIP-event timing inside the library (for benchmarks)."""

    @staticmethod
    def enable(on: bool = True):
        check(_lib().gal_timing_enable(1 if on else 0), "gal_timing_enable")

    @staticmethod
    def reset():
        check(_lib().gal_timing_reset(), "gal_timing_reset")

    @staticmethod
    def read() -> dict:
        """{kernel name: (total ms, launches)}; synchronises."""
        n = _lib().gal_timing_read(0, None, None, None)
        if n < 0:
            check(n, "gal_timing_read")
        names = (ctypes.c_char_p * max(n, 1))()
        ms = (ctypes.c_double * max(n, 1))()
        cnt = (ctypes.c_int64 * max(n, 1))()
        n = _lib().gal_timing_read(n, names, ms, cnt)
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(n)}


def probe_stage_bytes(blocks: int) -> int:
    """Workspace bytes of the stage-handoff probe (gal_probe_stage_bytes)."""
    return int(_lib().gal_probe_stage_bytes(blocks))


def probe_stage(mode: int, blocks: int, ws: torch.Tensor):
    """One launch of the stage-handoff probe (gal_probe_stage) on the current
    stream: every block writes 8 KB, then one agent-scope atomic per block --
    none (0), relaxed (1), release (2) or acquire-release (3)."""
    check(_lib().gal_probe_stage(mode, blocks, _ptr(ws), ws.numel() * ws.element_size(),
                                 _stream(ws.device)), "gal_probe_stage")


# ----------------------------------------------------------------------------
# autograd: chi^2 of a profile / image on a dataset, differentiable in the model
class _Chi2Profile(torch.autograd.Function):
    @staticmethod
    def forward(ctx, I, ds, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec):
        c2, g = ds.chi2Profile_grad(I.detach().contiguous(), Rmin, dR, Nxy, dxy, inc, PA, dRA,
                                    dDec)
        ctx.save_for_backward(g)
        return c2

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return (gout.to(g.dtype) * g,) + (None,) * 9


class _Chi2Image(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image, ds, dxy, PA, dRA, dDec, inc):
        c2, g = ds.chi2Image_grad(image.detach().contiguous(), dxy, PA, dRA, dDec, inc)
        ctx.save_for_backward(g)
        return c2

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return (gout.to(g.dtype) * g,) + (None,) * 6


def chi2_profile(ds: "Dataset", I, Rmin, dR, Nxy, dxy, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0):
    """Differentiable chi^2 of a radial profile on a dataset (d/dI by the adjoint)."""
    return _Chi2Profile.apply(I, ds, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec)


def chi2_image(ds: "Dataset", image, dxy, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0):
    """Differentiable chi^2 of an image on a dataset (d/dimage by the adjoint)."""
    return _Chi2Image.apply(image, ds, dxy, PA, dRA, dDec, inc)


_load_tune_cache()
