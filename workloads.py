"""Seeded synthetic inputs for the visibility / chi-square path.

This module only draws inputs: uv coverages, model images and profiles, noise.
It holds none of the method's arithmetic (no transform, no sampling, no
chi-square), so both the oracle-side tests and the GPU side may use it.
Observed visibilities are assembled by the caller as ``model + noise`` from
whichever model it trusts (the oracle in tests, the library in the benchmark).

The workloads stand in for the paper's unspecified profiles, images and uv
sets: their sizes follow the paper's timing setup (M = 10^6, FP64, images
512^2 ... 16384^2, Sec. 6) and its table of ALMA / VLA configurations
(Sec. 3.4, Table tb:array.config.matrix.properties, lambda = 1.3 mm).

Units: angles in radians, uv in wavelengths, profiles in Jy/sr, images in
Jy/pixel, weights 1/sigma^2 in Jy^-2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ARCSEC = math.pi / 648000.0
DEG = math.pi / 180.0


# ----------------------------------------------------------------------------
# uv coverages
# ----------------------------------------------------------------------------
def uv_uniform_disk(M: int, radius: float, seed: int):
    """M points uniform in a disk: rho = R sqrt(U), phi = 2 pi U'."""
    rng = np.random.default_rng(seed)
    rho = radius * np.sqrt(rng.random(M))
    phi = 2.0 * np.pi * rng.random(M)
    return rho * np.cos(phi), rho * np.sin(phi)


def uv_log_uniform(M: int, rho_min: float, rho_max: float, seed: int):
    """M points with ln(rho) uniform in [ln rho_min, ln rho_max], uniform angle."""
    rng = np.random.default_rng(seed)
    rho = np.exp(rng.uniform(math.log(rho_min), math.log(rho_max), M))
    phi = 2.0 * np.pi * rng.random(M)
    return rho * np.cos(phi), rho * np.sin(phi)


def noise(M: int, sigma: float, seed: int):
    """Independent N(0, sigma^2) draws for the real and imaginary parts, and w = 1/sigma^2."""
    rng = np.random.default_rng(seed)
    nre = rng.normal(0.0, sigma, M)
    nim = rng.normal(0.0, sigma, M)
    w = np.full(M, 1.0 / sigma**2)
    return nre, nim, w


# ----------------------------------------------------------------------------
# model images and profiles
# ----------------------------------------------------------------------------
def pixel_axes(N: int, dxy: float):
    """Sky coordinates of the pixel centres: x_c = (N/2 - c) dxy (East at c = 0),
    y_r = (N/2 - r) dxy (North at r = 0); the paper's image orientation (Sec. 2.2)."""
    idx = np.arange(N, dtype=np.float64)
    return (N // 2 - idx) * dxy, (N // 2 - idx) * dxy


def gaussian_image(N: int, dxy: float, flux: float, sigma_x: float, sigma_y: float,
                   x0: float = 0.0, y0: float = 0.0, angle: float = 0.0):
    """Pixel values F dxy^2 / (2 pi sx sy) exp(-x'^2/2sx^2 - y'^2/2sy^2), the
    Gaussian centred at (x0, y0) with axes rotated by ``angle``."""
    x, y = pixel_axes(N, dxy)
    X = x[None, :] - x0
    Y = y[:, None] - y0
    ca, sa = math.cos(angle), math.sin(angle)
    xr = X * ca + Y * sa
    yr = -X * sa + Y * ca
    amp = flux * dxy * dxy / (2.0 * math.pi * sigma_x * sigma_y)
    return amp * np.exp(-0.5 * (xr / sigma_x) ** 2 - 0.5 * (yr / sigma_y) ** 2)


def blob_image(N: int, dxy: float, n_blobs: int, seed: int, total_flux: float = 1.0):
    """Sum of elliptical Gaussian blobs: centres uniform in |x|,|y| <= N dxy / 4,
    sigma log-uniform in [2, 16] px, axis ratio U[0.5, 1], orientation U[0, pi),
    fluxes log-normal(0, 1) renormalised to ``total_flux``.  Each blob is
    evaluated inside a +-8 sigma box (the rest is below 1e-13 of its peak)."""
    rng = np.random.default_rng(seed)
    half = N * dxy / 4.0
    cx = rng.uniform(-half, half, n_blobs)
    cy = rng.uniform(-half, half, n_blobs)
    sig = np.exp(rng.uniform(math.log(2.0), math.log(16.0), n_blobs)) * dxy
    ratio = rng.uniform(0.5, 1.0, n_blobs)
    ang = rng.uniform(0.0, math.pi, n_blobs)
    flux = rng.lognormal(0.0, 1.0, n_blobs)
    flux *= total_flux / flux.sum()
    img = np.zeros((N, N), dtype=np.float64)
    x, y = pixel_axes(N, dxy)
    for b in range(n_blobs):
        sx, sy = sig[b], sig[b] * ratio[b]
        box = int(math.ceil(8.0 * sx / dxy)) + 1
        c0 = int(round(N // 2 - cx[b] / dxy))
        r0 = int(round(N // 2 - cy[b] / dxy))
        cs = slice(max(c0 - box, 0), min(c0 + box + 1, N))
        rs = slice(max(r0 - box, 0), min(r0 + box + 1, N))
        X = x[cs][None, :] - cx[b]
        Y = y[rs][:, None] - cy[b]
        ca, sa = math.cos(ang[b]), math.sin(ang[b])
        xr = X * ca + Y * sa
        yr = -X * sa + Y * ca
        amp = flux[b] * dxy * dxy / (2.0 * math.pi * sx * sy)
        img[rs, cs] += amp * np.exp(-0.5 * (xr / sx) ** 2 - 0.5 * (yr / sy) ** 2)
    return img


def gapped_powerlaw_profile(r_arcsec, gaps=((0.3, 0.02, 0.9), (0.7, 0.04, 0.7))):
    """I(r) ~ r^-0.8 exp(-(r / 1'')^2) prod_g [1 - depth_g exp(-(r - r_g)^2 / (2 w_g^2))],
    r in arcsec, gaps given as (centre, width, depth) in arcsec."""
    r = np.asarray(r_arcsec, dtype=np.float64)
    with np.errstate(divide="ignore"):
        base = np.where(r > 0, r, np.inf) ** -0.8 * np.exp(-(r / 1.0) ** 2)
    for rg, wg, dg in gaps:
        base = base * (1.0 - dg * np.exp(-((r - rg) ** 2) / (2.0 * wg**2)))
    return base


def _face_on_flux(profile_fn, r_max_arcsec: float) -> float:
    """2 pi int_0^rmax I(r) r dr (r in radians) for a profile in arbitrary units,
    by the trapezoid rule on a fine grid in sqrt(r) (the integrand ~ r^0.2 near 0)."""
    s = np.linspace(0.0, math.sqrt(r_max_arcsec), 400001)
    r = s * s
    f = np.zeros_like(r)
    f[1:] = profile_fn(r[1:]) * r[1:] * 2.0 * s[1:]  # I(r) r dr/ds
    return 2.0 * math.pi * np.trapezoid(f, s) * ARCSEC**2


# ----------------------------------------------------------------------------
# the benchmark / parity workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    kind: str                    # "image" or "profile"
    N: int
    dxy: float
    u: np.ndarray
    v: np.ndarray
    noise_re: np.ndarray
    noise_im: np.ndarray
    w: np.ndarray
    PA: float = 0.0
    inc: float = 0.0
    dRA: float = 0.0
    dDec: float = 0.0
    image: np.ndarray | None = None
    I: np.ndarray | None = None
    Rmin: float = 0.0
    dR: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.u.size)


def gaussian_image_256() -> Workload:
    """chi2Image, 256^2 FP64: elliptical Gaussian (1 Jy, sigma 0.2'' N-S and
    0.2'' cos 30 deg E-W, i.e. a 30 deg inclination in the image itself),
    dxy = 0.01'', M = 10^4 uniform in a disk of radius 0.4 / dxy,
    PA = 60 deg, dRA = dDec = 0.05'', noise sigma 1e-3 Jy."""
    N, dxy = 256, 0.01 * ARCSEC
    sig = 0.2 * ARCSEC
    img = gaussian_image(N, dxy, 1.0, sig * math.cos(30 * DEG), sig)
    u, v = uv_uniform_disk(10_000, 0.4 / dxy, seed=1000)
    nre, nim, w = noise(u.size, 1e-3, seed=1001)
    return Workload("gaussian_chi2Image_256_M1e4", "image", N, dxy, u, v, nre, nim, w,
                    PA=60 * DEG, inc=0.0, dRA=0.05 * ARCSEC, dDec=0.05 * ARCSEC, image=img,
                    meta={"image_inclination_deg": 30.0})


def gapped_profile(Nr: int = 4096):
    """The gapped power-law profile in Jy/sr, normalised to a
    face-on flux of 1 Jy, on r_j = Rmin + j dR out to 5.4''."""
    Rmin_as = 1e-4
    Rmax_as = 5.4
    dR_as = (Rmax_as - Rmin_as) / (Nr - 1)
    r_as = Rmin_as + dR_as * np.arange(Nr)
    norm = _face_on_flux(gapped_powerlaw_profile, Rmax_as)
    I = gapped_powerlaw_profile(r_as) / norm
    return I, Rmin_as * ARCSEC, dR_as * ARCSEC


def profile_2048(M: int = 1_000_000) -> Workload:
    """chi2Profile, 2048^2 FP64: Nr = 4096 profile, dxy = 0.003'', M = 10^6
    uv points log-uniform in [1.877e5, 1.2457e7] lambda (ALMA C43-10 at
    1.3 mm), inc = 45 deg, PA = 120 deg, noise sigma 1e-3 Jy."""
    N, dxy = 2048, 0.003 * ARCSEC
    I, Rmin, dR = gapped_profile()
    u, v = uv_log_uniform(M, 1.877e5, 1.2457e7, seed=1100)
    nre, nim, w = noise(u.size, 1e-3, seed=1101)
    return Workload("gapped_chi2Profile_2048_M1e6", "profile", N, dxy, u, v, nre, nim, w,
                    PA=120 * DEG, inc=45 * DEG, I=I, Rmin=Rmin, dR=dR)


def ring_image(N: int, dxy: float, flux: float, r0: float, width: float, inc: float,
               phi0: float, phi_sigma: float):
    """Gaussian ring of radius r0 and Gaussian width ``width`` (rad), inclined
    by ``inc`` (x stretched by 1 / cos inc before the radius is taken),
    modulated in azimuth by exp(-(phi - phi0)^2 / (2 phi_sigma^2)) (phi the
    position angle East of North of the deprojected point, the difference
    wrapped into [-pi, pi)), pixel values summing to ``flux``."""
    x, y = pixel_axes(N, dxy)
    X = x[None, :] / math.cos(inc)
    Y = y[:, None]
    rho = np.hypot(X, Y)
    phi = np.arctan2(X, Y)
    dphi = (phi - phi0 + math.pi) % (2.0 * math.pi) - math.pi
    img = np.exp(-0.5 * ((rho - r0) / width) ** 2 - 0.5 * (dphi / phi_sigma) ** 2)
    return img * (flux / img.sum())


def spectral_cube(n_chan: int = 64, N: int = 1024, M_range=(200_000, 1_000_000),
                  seed: int = 1300):
    """Channels of a spectral cube at N^2 FP32 (64 at 1024^2), dxy = 0.054''
    (ALMA C43-4 row of the paper's table).  One base uv set of 10^6 points,
    log-uniform radius over the C43-4 baselines at 1.3 mm; channel c scales it
    by its frequency ratio s_c = 1 + 0.05 c / (n - 1) and keeps the first
    M_c = round(M_lo + (M_hi - M_lo) U_c) points of its own permutation
    (ragged).  Its image is a Gaussian ring (r0 = 2'', width 0.5'', inclined
    40 deg) modulated in azimuth around 2 pi c / 64 (sigma 0.4 rad), 0.1 Jy;
    noise sigma 1e-3 Jy.  Yields one Workload per channel."""
    dxy = 0.054 * ARCSEC
    rho_lo, rho_hi = 14.6 / 1.3e-3, 783.5 / 1.3e-3
    u0, v0 = uv_log_uniform(M_range[1], rho_lo, rho_hi, seed=seed - 1)
    for k in range(n_chan):
        rng = np.random.default_rng(seed + k)
        f = 1.0 + 0.05 * k / max(n_chan - 1, 1)
        M = int(round(M_range[0] + (M_range[1] - M_range[0]) * rng.random()))
        sel = rng.permutation(u0.size)[:M]
        nre, nim, w = noise(M, 1e-3, seed=seed + 100 + k)
        img = ring_image(N, dxy, 0.1, 2.0 * ARCSEC, 0.5 * ARCSEC, 40 * DEG,
                         2.0 * math.pi * k / 64.0, 0.4)
        yield Workload(f"cube_chan{k}_N{N}_M{M}", "image", N, dxy, u0[sel] * f, v0[sel] * f, nre,
                       nim, w, PA=30 * DEG, inc=0.0, dRA=0.0, dDec=0.0, image=img)


# pixel sizes of the paper's table (ALMA at 1.3 mm) for the image sizes it lists
TABLE_DXY = {512: 0.108 * ARCSEC, 1024: 0.054 * ARCSEC, 2048: 0.027 * ARCSEC,
             4096: 0.013 * ARCSEC}


def mixed_models(n: int = 32, sizes=(512, 1024, 2048, 4096), M_range=(100_000, 2_000_000),
                 seed: int = 1400):
    """Models of mixed sizes, each on its own observation: model i draws Nxy
    uniformly from ``sizes`` with the table's pixel size, an image of 20
    Gaussian blobs (as blobs_4096), M_i log-uniform in M_range, uv radius
    log-uniform in [rho_max / 100, rho_max] with rho_max = 1 / (5 dxy) (the
    grid reaches f_max = 2.5 times it), uniform angle, noise sigma 1e-3 Jy,
    random PA and offsets (seeds 1400 + i).  Yields one Workload per model."""
    for i in range(n):
        rng = np.random.default_rng(seed + i)
        N = int(rng.choice(sizes))
        dxy = TABLE_DXY[N]
        M = int(round(math.exp(rng.uniform(math.log(M_range[0]), math.log(M_range[1])))))
        rho_max = 1.0 / (5.0 * dxy)
        u, v = uv_log_uniform(M, rho_max / 100.0, rho_max, seed=seed + 100 + i)
        nre, nim, w = noise(M, 1e-3, seed=seed + 200 + i)
        img = blob_image(N, dxy, 20, seed=seed + 300 + i)
        yield Workload(f"mixed{i}_N{N}_M{M}", "image", N, dxy, u, v, nre, nim, w,
                       PA=rng.uniform(0.0, math.pi), inc=0.0,
                       dRA=float(rng.normal(0.0, 2 * dxy)), dDec=float(rng.normal(0.0, 2 * dxy)),
                       image=img)


def field_of_copies(c: Workload, n: int, seed: int) -> list:
    """A field of n copies of the profile workload ``c``: the first at c's own
    geometry, the others (sharing its spectrum) at random PA and offsets of up
    to 1'' from the phase centre.  Source dicts as the oracle takes them."""
    rng = np.random.default_rng(seed)
    out = [dict(kind="profile", I=c.I, Rmin=c.Rmin, dR=c.dR, Nxy=c.N, dxy=c.dxy, inc=c.inc,
                PA=c.PA, dRA=c.dRA, dDec=c.dDec)]
    for _ in range(n - 1):
        out.append(dict(kind="profile", I=None, share=0, dxy=c.dxy, Nxy=c.N,
                        PA=rng.uniform(0.0, math.pi),
                        dRA=rng.uniform(-1.0, 1.0) * ARCSEC, dDec=rng.uniform(-1.0, 1.0) * ARCSEC))
    return out


def image_2048(M: int = 1_000_000) -> Workload:
    """chi2Image at the headline size, 2048^2 FP64: 200 Gaussian blobs (as
    blobs_4096) at dxy = 0.003'', on the uv set and noise of profile_2048
    (M = 1e6, C43-10), PA = 120 deg, inc = 45 deg (deprojection of the uv),
    offsets 0.01''."""
    N, dxy = 2048, 0.003 * ARCSEC
    img = blob_image(N, dxy, 200, seed=1250)
    u, v = uv_log_uniform(M, 1.877e5, 1.2457e7, seed=1100)
    nre, nim, w = noise(u.size, 1e-3, seed=1101)
    return Workload("blobs_chi2Image_2048_M1e6", "image", N, dxy, u, v, nre, nim, w,
                    PA=120 * DEG, inc=45 * DEG, dRA=0.01 * ARCSEC, dDec=0.01 * ARCSEC, image=img)


def blobs_4096(M: int = 5_000_000) -> Workload:
    """chi2Image, 4096^2: 200 Gaussian blobs, dxy = 0.013'' (ALMA C43-6),
    M = 5e6 log-uniform in [1.123e4, 1.936e6] lambda, noise sigma 1e-3 Jy."""
    N, dxy = 4096, 0.013 * ARCSEC
    img = blob_image(N, dxy, 200, seed=1200)
    u, v = uv_log_uniform(M, 1.123e4, 1.936e6, seed=1201)
    nre, nim, w = noise(u.size, 1e-3, seed=1202)
    return Workload("blobs_chi2Image_4096_M5e6", "image", N, dxy, u, v, nre, nim, w,
                    PA=0.0, inc=0.0, image=img)


# ----------------------------------------------------------------------------
# small random cases for parity sweeps
# ----------------------------------------------------------------------------
def random_case(N: int, M: int, seed: int, kind: str = "image", fill: float = 0.9,
                Nr: int | None = None) -> Workload:
    """Random image (or profile), uv inside ``fill`` of the valid radius
    (N/2 - 1) du, random PA / inc / offsets, noise sigma 1e-3."""
    rng = np.random.default_rng(seed)
    dxy = 0.01 * ARCSEC * (1.0 + rng.random())
    du = 1.0 / (N * dxy)
    rho_lim = fill * (N / 2 - 1) * du
    u, v = uv_uniform_disk(M, rho_lim, seed=seed + 1)
    nre, nim, w = noise(M, 1e-3, seed=seed + 2)
    w = w * rng.uniform(0.5, 1.5, M)
    PA = rng.uniform(0.0, 2 * math.pi)
    inc = rng.uniform(0.0, 70 * DEG)
    dRA, dDec = rng.normal(0.0, 5 * dxy, 2)
    if kind == "image":
        img = rng.normal(0.0, 1e-3, (N, N)) + gaussian_image(
            N, dxy, 1.0, 3 * dxy, 2 * dxy, x0=2 * dxy, y0=-3 * dxy, angle=0.3)
        return Workload(f"random_image_N{N}_M{M}_s{seed}", "image", N, dxy, u, v, nre, nim, w,
                        PA=PA, inc=inc, dRA=dRA, dDec=dDec, image=img)
    Nr = Nr or max(2, N)
    Rmin = 0.1 * dxy * rng.random()
    Rmax = 0.75 * N * dxy
    dR = (Rmax - Rmin) / (Nr - 1)
    r = Rmin + dR * np.arange(Nr)
    I = np.exp(-((r / (0.15 * N * dxy)) ** 2)) * (1.0 + 0.3 * rng.random(Nr)) / dxy**2
    return Workload(f"random_profile_N{N}_M{M}_s{seed}", "profile", N, dxy, u, v, nre, nim, w,
                    PA=PA, inc=inc, dRA=dRA, dDec=dDec, I=I, Rmin=Rmin, dR=dR)


# ----------------------------------------------------------------------------
# served load: 8 resident datasets and a Poisson stream of profile requests
SERVE_DXY = 1.0 / (2.0 * 2.5e6)   # rad: f_max = 2.5 at rho_max = 1e6 lambda for every N


def serve_datasets(n: int = 8, M_range=(100_000, 2_000_000), seed0: int = 1500):
    """Datasets d: M_d log-uniform in M_range, uv log-uniform radius in
    [2e4, 1e6] lambda, noise sigma 1e-3 (observed = model + noise, the model
    supplied by the caller)."""
    out = []
    for d in range(n):
        rng = np.random.default_rng(seed0 + d)
        M = int(round(math.exp(rng.uniform(math.log(M_range[0]), math.log(M_range[1])))))
        u, v = uv_log_uniform(M, 2e4, 1e6, seed=seed0 + 100 + d)
        nre, nim, w = noise(M, 1e-3, seed=seed0 + 200 + d)
        out.append({"name": f"d{d}", "u": u, "v": v, "noise_re": nre, "noise_im": nim, "w": w})
    return out


def serve_requests(n: int, seed: int, n_datasets: int = 8, sizes=(512, 1024, 2048)):
    """Request parameters: dataset uniform, Nxy uniform in ``sizes`` ({512,
    1024, 2048}), Nr in U{512..4096}, a gapped power-law profile with random
    gap positions and depths, Rmin = 1e-4 N dxy, R_max = 1.05 (N/2) dxy
    sqrt(1/cos^2 i + 1), inc ~ U[0, 70 deg], PA ~ U[0, 180 deg), offsets
    ~ N(0, (5 dxy)^2)."""
    rng = np.random.default_rng(seed)
    dxy = SERVE_DXY
    reqs = []
    for _ in range(n):
        d = int(rng.integers(0, n_datasets))
        N = int(rng.choice(list(sizes)))
        Nr = int(rng.integers(512, 4097))
        inc = rng.uniform(0.0, 70.0) * DEG
        PA = rng.uniform(0.0, 180.0) * DEG
        dRA, dDec = rng.normal(0.0, 5 * dxy, 2)
        Rmin = 1e-4 * N * dxy
        Rmax = 1.05 * (N / 2) * dxy * math.sqrt(1.0 / math.cos(inc) ** 2 + 1.0)
        dR = (Rmax - Rmin) / (Nr - 1)
        r_as = (Rmin + dR * np.arange(Nr)) / ARCSEC
        scale = (N / 2) * dxy / ARCSEC / 5.0            # profile scale relative to the field
        gaps = ((rng.uniform(0.2, 0.8) * scale, 0.02 * scale, rng.uniform(0.3, 0.9)),
                (rng.uniform(0.2, 0.8) * scale, 0.04 * scale, rng.uniform(0.3, 0.9)))
        I = gapped_powerlaw_profile(r_as / scale, gaps=tuple((g[0] / scale, g[1] / scale, g[2])
                                                              for g in gaps)) * 1e10
        reqs.append({"dataset": f"d{d}", "I": I, "Rmin": Rmin, "dR": dR, "Nxy": N, "dxy": dxy,
                     "inc": inc, "PA": PA, "dRA": float(dRA), "dDec": float(dDec)})
    return reqs
