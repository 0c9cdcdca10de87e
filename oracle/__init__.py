"""FP64 CPU oracle for the visibility / chi-square path of GALARIO
(Tazzari, Beaujean & Testi 2018, arXiv:1709.06999).

TEST INFRASTRUCTURE ONLY.  The oracle is the independent checker of the HIP
library: it shares no code with it, and only ``tests/``, the smoke entry and the
CPU-baseline leg of the benchmark may import it.  The product path never calls
it.  The arithmetic lives in ``oracle.c`` (plain C + OpenMP, FP64, direct DFT);
this module only marshals numpy arrays.

Sign convention.  The paper's body text (Sec. 3.1, Eq. complex.visibility.obs.xy;
Sec. 3.3 translation) writes V = FT with exp(-2 pi i (u l + v m)) and a phase
exp(-2 pi i (u dRA + v dDec)); its Appendix D reference functions, which fix
the pixel orientation (East left, North up) jointly with the transform, compute
V(u, v) = sum_pixels I exp(+2 pi i (u x + v y)) with the offset phase
exp(+i theta), theta = 2 pi (u dRA + v dDec).  The two differ by complex
conjugation.  The oracle (and the library) follow Appendix D.

Functions and the passages they follow:
  sweep          Sec. 2.2 (sampleProfile, inc), Sec. 4 (Create image), App. D
  grid           Sec. 4 (shift -> real-to-complex FFT -> shift) as a direct DFT
  grid_cell      one node of ``grid`` by the non-separable double sum
  sample_grid    Sec. 3.3 (rotation by PA, translation), Sec. 3.4 (bilinear), App. D
  sample_direct  as sample_grid with every node from ``grid_cell``
  chi2           Sec. 3.1, Eq. def.chi.square
  grad_image / grad_profile   transpose of the above (not in the paper)
  sample_sources / chi2_sources / grad_sources   Sec. 3.2 (a field of several
                 sources is the sum of their visibilities), on the above
  get_image_size Sec. 3.4, criteria (i), (iia), (iib)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def build() -> str:
    """Compile oracle.c with gcc (FP64, OpenMP, no fast-math)."""
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_sweep.argtypes = [_D, _I64, ctypes.c_double, ctypes.c_double, _I64,
                              ctypes.c_double, ctypes.c_double, _D]
    lib.orc_sweep.restype = ctypes.c_int
    lib.orc_grid.argtypes = [_D, _I64, _D]
    lib.orc_grid.restype = ctypes.c_int
    lib.orc_grid_cell.argtypes = [_D, _I64, _I64, _I64, _D]
    lib.orc_grid_cell.restype = None
    for name in ("orc_sample", "orc_sample_direct"):
        f = getattr(lib, name)
        f.argtypes = [_D, _I64, ctypes.c_double, _D, _D, _I64, ctypes.c_double,
                      ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        f.restype = _I64
    lib.orc_chi2.argtypes = [_D, _D, _D, _D, _I64]
    lib.orc_chi2.restype = ctypes.c_double
    lib.orc_grad_image.argtypes = [_D, _I64, ctypes.c_double, _D, _D, _D, _D, _D,
                                   _I64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, _D]
    lib.orc_grad_image.restype = _I64
    lib.orc_grad_profile.argtypes = [_D, _I64, ctypes.c_double, ctypes.c_double,
                                     _I64, ctypes.c_double, ctypes.c_double, _D]
    lib.orc_grad_profile.restype = ctypes.c_int
    lib.orc_sweep_dinc.argtypes = lib.orc_sweep.argtypes
    lib.orc_sweep_dinc.restype = ctypes.c_int
    lib.orc_geograd.argtypes = [_D, _D, _I64, ctypes.c_double, _D, _D, _D, _D, _D, _I64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, _D]
    lib.orc_geograd.restype = _I64
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for later oracle calls (n < 1: all cores); timing only."""
    _load().orc_set_num_threads(int(n))


def sweep(I, Rmin, dR, N, dxy, inc=0.0) -> np.ndarray:
    """Image [N, N] in Jy/pixel from the radial profile I [Jy/sr]."""
    I = _f64(I)
    img = np.empty((int(N), int(N)), dtype=np.float64)
    rc = _load().orc_sweep(_p(I), I.size, float(Rmin), float(dR), int(N), float(dxy),
                           float(inc), _p(img))
    if rc != 0:
        raise ValueError(f"orc_sweep: error {rc}")
    return img


def grid(img) -> np.ndarray:
    """Half spectrum G [N, N/2+1] (complex128), rows p unshifted (frequency p - N [p >= N/2])."""
    img = _f64(img)
    N = img.shape[0]
    assert img.shape == (N, N)
    G = np.empty((N, N // 2 + 1, 2), dtype=np.float64)
    rc = _load().orc_grid(_p(img), N, _p(G))
    if rc != 0:
        raise ValueError(f"orc_grid: error {rc}")
    return G[..., 0] + 1j * G[..., 1]


def grid_cell(img, p, q) -> complex:
    img = _f64(img)
    out = np.empty(2, dtype=np.float64)
    _load().orc_grid_cell(_p(img), img.shape[0], int(p), int(q), _p(out))
    return complex(out[0], out[1])


def sample_grid(G, N, dxy, u, v, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0) -> np.ndarray:
    """Sample a half spectrum from ``grid`` at the uv points (NaN where off grid)."""
    G = np.ascontiguousarray(G, dtype=np.complex128)
    Gi = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1))
    u, v = _f64(u), _f64(v)
    out = np.empty((u.size, 2), dtype=np.float64)
    _load().orc_sample(_p(Gi), int(N), float(dxy), _p(u), _p(v), u.size, float(PA),
                       float(dRA), float(dDec), float(inc), _p(out))
    return out[:, 0] + 1j * out[:, 1]


def sample_direct(img, dxy, u, v, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0) -> np.ndarray:
    """Like sampleImage, each node by the non-separable double sum (few points, any N)."""
    img = _f64(img)
    u, v = _f64(u), _f64(v)
    out = np.empty((u.size, 2), dtype=np.float64)
    _load().orc_sample_direct(_p(img), img.shape[0], float(dxy), _p(u), _p(v), u.size,
                              float(PA), float(dRA), float(dDec), float(inc), _p(out))
    return out[:, 0] + 1j * out[:, 1]


def sampleImage(image, dxy, u, v, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0) -> np.ndarray:
    image = _f64(image)
    return sample_grid(grid(image), image.shape[0], dxy, u, v, PA, dRA, dDec, inc)


def sampleProfile(I, Rmin, dR, Nxy, dxy, u, v, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0) -> np.ndarray:
    img = sweep(I, Rmin, dR, Nxy, dxy, inc)
    return sample_grid(grid(img), Nxy, dxy, u, v, PA, dRA, dDec, 0.0)


def chi2(V, re, im, w) -> float:
    V = np.ascontiguousarray(V, dtype=np.complex128)
    Vi = np.ascontiguousarray(np.stack([V.real, V.imag], axis=-1))
    re, im, w = _f64(re), _f64(im), _f64(w)
    return float(_load().orc_chi2(_p(Vi), _p(re), _p(im), _p(w), re.size))


def chi2Image(image, dxy, u, v, re, im, w, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0) -> float:
    return chi2(sampleImage(image, dxy, u, v, PA, dRA, dDec, inc), re, im, w)


def chi2Profile(I, Rmin, dR, Nxy, dxy, u, v, re, im, w, inc=0.0, PA=0.0, dRA=0.0,
                dDec=0.0) -> float:
    return chi2(sampleProfile(I, Rmin, dR, Nxy, dxy, u, v, inc, PA, dRA, dDec), re, im, w)


def grad_image(image, dxy, u, v, re, im, w, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0):
    """(chi2, d chi2 / d image) -- the transpose of the sampling map."""
    image = _f64(image)
    N = image.shape[0]
    V = sampleImage(image, dxy, u, v, PA, dRA, dDec, inc)
    Vi = np.ascontiguousarray(np.stack([V.real, V.imag], axis=-1))
    u, v, re, im, w = map(_f64, (u, v, re, im, w))
    g = np.empty((N, N), dtype=np.float64)
    _load().orc_grad_image(_p(Vi), N, float(dxy), _p(u), _p(v), _p(re), _p(im), _p(w),
                           u.size, float(PA), float(dRA), float(dDec), float(inc), _p(g))
    return chi2(V, re, im, w), g


def grad_profile(I, Rmin, dR, Nxy, dxy, u, v, re, im, w, inc=0.0, PA=0.0, dRA=0.0, dDec=0.0):
    """(chi2, d chi2 / d I) through the sweep."""
    I = _f64(I)
    img = sweep(I, Rmin, dR, Nxy, dxy, inc)
    c2, gimg = grad_image(img, dxy, u, v, re, im, w, PA, dRA, dDec, 0.0)
    gI = np.empty(I.size, dtype=np.float64)
    rc = _load().orc_grad_profile(_p(np.ascontiguousarray(gimg)), I.size, float(Rmin),
                                  float(dR), int(Nxy), float(dxy), float(inc), _p(gI))
    if rc != 0:
        raise ValueError(f"orc_grad_profile: error {rc}")
    return c2, gI


def sweep_dinc(I, Rmin, dR, N, dxy, inc=0.0) -> np.ndarray:
    """d image / d inc of the swept profile (orc_sweep_dinc)."""
    I = _f64(I)
    out = np.empty((N, N), dtype=np.float64)
    rc = _load().orc_sweep_dinc(_p(I), I.size, float(Rmin), float(dR), int(N), float(dxy),
                                float(inc), _p(out))
    if rc != 0:
        raise ValueError(f"orc_sweep_dinc: error {rc}")
    return out


def _geograd(G, Gt, N, dxy, u, v, re, im, w, PA, dRA, dDec, inc):
    u, v, re, im, w = map(_f64, (u, v, re, im, w))
    Gi = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1))
    Gti = None if Gt is None else np.ascontiguousarray(np.stack([Gt.real, Gt.imag], axis=-1))
    out = np.empty(5, dtype=np.float64)
    _load().orc_geograd(_p(Gi), None if Gti is None else _p(Gti), int(N), float(dxy), _p(u),
                        _p(v), _p(re), _p(im), _p(w), u.size, float(PA), float(dRA),
                        float(dDec), float(inc), _p(out))
    return float(out[0]), out[1:].copy()


def geograd_image(image, dxy, u, v, re, im, w, PA=0.0, dRA=0.0, dDec=0.0, inc=0.0):
    """(chi2, [d/dPA, d/d dRA, d/d dDec, d/d inc]) of chi2Image (orc_geograd)."""
    image = _f64(image)
    return _geograd(grid(image), None, image.shape[0], dxy, u, v, re, im, w, PA, dRA, dDec, inc)


def geograd_profile(I, Rmin, dR, Nxy, dxy, u, v, re, im, w, inc=0.0, PA=0.0, dRA=0.0,
                    dDec=0.0):
    """(chi2, [d/dPA, d/d dRA, d/d dDec, d/d inc]) of chi2Profile: the inclination
    derivative samples the transform of sweep_dinc's image."""
    G = grid(sweep(I, Rmin, dR, Nxy, dxy, inc))
    Gt = grid(sweep_dinc(I, Rmin, dR, Nxy, dxy, inc))
    return _geograd(G, Gt, Nxy, dxy, u, v, re, im, w, PA, dRA, dDec, inc)


def _resolve(sources):
    """Source dicts with every shared spectrum spelled out: a source with
    "share": k uses the model of source k, and for a profile also its Rmin, dR,
    Nxy, dxy and inc (those make the transform); its PA and offsets (and inc,
    for an image) stay its own."""
    out = []
    for s in sources:
        k = s.get("share")
        if k is None:
            out.append(s)
            continue
        o = sources[k]
        r = dict(s)
        keys = ("image", "dxy") if s["kind"] == "image" else ("I", "Rmin", "dR", "Nxy", "dxy", "inc")
        for key in keys:
            r[key] = o[key]
        out.append(r)
    return out


def _source_vis(sources, u, v):
    """Each source's visibilities.  A source samples the half spectrum of its
    own model -- for an image, with its inclination applied at sampling; for
    a profile, the transform of the inclined swept image (as sampleImage and
    sampleProfile) -- and a source with "share" samples its owner's, which is
    transformed once."""
    res = _resolve(sources)
    spectra = {}
    out = []
    for i, s in enumerate(res):
        owner = sources[i].get("share")
        owner = i if owner is None else owner
        if owner not in spectra:
            o = res[owner]
            img = o["image"] if o["kind"] == "image" else sweep(
                o["I"], o["Rmin"], o["dR"], o["Nxy"], o["dxy"], o.get("inc", 0.0))
            spectra[owner] = (grid(img), np.shape(img)[0])
        G, N = spectra[owner]
        inc = s.get("inc", 0.0) if s["kind"] == "image" else 0.0
        out.append(sample_grid(G, N, s["dxy"], u, v, s.get("PA", 0.0), s.get("dRA", 0.0),
                               s.get("dDec", 0.0), inc))
    return out


def sample_sources(sources, u, v) -> np.ndarray:
    """Visibilities of a field of several sources (Sec. 3.2: the sources'
    visibilities add up, each source placed by its own phase shift).
    ``sources``: dicts {"kind": "image", "image", "dxy", PA, dRA, dDec, inc}
    or {"kind": "profile", "I", "Rmin", "dR", "Nxy", "dxy", inc, PA, dRA,
    dDec} (geometry keys default to 0), optionally "share": k (see _resolve)."""
    V = np.zeros(np.size(u), dtype=np.complex128)
    for Vs in _source_vis(sources, u, v):
        V += Vs
    return V


def chi2_sources(sources, u, v, re, im, w) -> float:
    """chi^2 of the summed model (Eq. def.chi.square on sample_sources)."""
    return chi2(sample_sources(sources, u, v), re, im, w)


def grad_sources(sources, u, v, re, im, w):
    """(chi2, [d chi2 / d model of each source]) of the summed model.  With the
    other sources' visibilities moved to the observations, chi^2 is that of
    one source, so each gradient is grad_image / grad_profile against
    obs - V_others.  A source with "share" gets None: by the chain rule its
    gradient is added into the owner's."""
    res = _resolve(sources)
    Vs = _source_vis(sources, u, v)
    V = np.sum(Vs, axis=0)
    c2 = chi2(V, re, im, w)
    grads = [None] * len(sources)
    for i, s in enumerate(res):
        Vo = V - Vs[i]
        r_i, i_i = np.asarray(re) - Vo.real, np.asarray(im) - Vo.imag
        if s["kind"] == "image":
            _, g = grad_image(s["image"], s["dxy"], u, v, r_i, i_i, w, s.get("PA", 0.0),
                              s.get("dRA", 0.0), s.get("dDec", 0.0), s.get("inc", 0.0))
        else:
            _, g = grad_profile(s["I"], s["Rmin"], s["dR"], s["Nxy"], s["dxy"], u, v, r_i, i_i, w,
                                s.get("inc", 0.0), s.get("PA", 0.0), s.get("dRA", 0.0),
                                s.get("dDec", 0.0))
        owner = sources[i].get("share")
        owner = i if owner is None else owner
        grads[owner] = g if grads[owner] is None else grads[owner] + g
    return c2, grads


def get_image_size(u, v, PB=0.0, f_min=5.0, f_max=2.5, Gamma=0.6, smooth=False):
    """(N, dxy [rad]) for the uv points by the image-size criteria of Sec. 3.4.

    uv cell: criterion (iia), the image spans f_min times the largest
    recoverable scale Gamma / rho_min, so du = rho_min / (Gamma f_min); with a
    primary-beam FWHM PB > 0, criterion (iib), the image spans the beam, du =
    1 / PB.  Size: criterion (i), the grid reaches f_max times the longest
    baseline, N du / 2 >= f_max rho_max, with N the smallest power of two that
    does (the advice after the paper's table); smooth: the smallest even
    N = 2^a 3^b 5^c that does, found by trying every even N in turn.  Pixel:
    dxy = 1 / (N du), so the image keeps the field of (iia) or (iib) exactly."""
    rho = np.hypot(np.asarray(u, dtype=np.float64), np.asarray(v, dtype=np.float64))
    rho_min, rho_max = float(rho.min()), float(rho.max())
    du = 1.0 / PB if PB > 0 else rho_min / (Gamma * f_min)
    if smooth:
        def five_smooth(n):
            for f in (2, 3, 5):
                while n % f == 0:
                    n //= f
            return n == 1

        N = 2
        while N * du / 2.0 < f_max * rho_max or not five_smooth(N):
            N += 2
        return N, 1.0 / (N * du)
    N = 2
    while N * du / 2.0 < f_max * rho_max:
        N *= 2
    return N, 1.0 / (N * du)
