"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a brute-force sum written independently here, a library routine
(numpy FFT, scipy interpolators), or an invariant.  They are chosen so that a
dropped term, a wrong sign or index, or a transposed operand in the oracle
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy.interpolate import RectBivariateSpline, interp1d

import oracle
import workloads as wl

ARC = wl.ARCSEC


def _rng(seed):
    return np.random.default_rng(seed)


def _brute_grid(img):
    """sum_{r,c} img exp(-2 pi i (p (r - N/2) + q (c - N/2)) / N), written with
    numpy exponentials on the full index grid (no table, no separability)."""
    N = img.shape[0]
    r = np.arange(N) - N // 2
    p = np.arange(N)[:, None, None]
    q = np.arange(N // 2 + 1)[:, None]
    out = np.empty((N, N // 2 + 1), dtype=np.complex128)
    for pi in range(N):
        # phase[q, r, c]
        ph = np.exp(-2j * np.pi * (pi * r[None, :, None] + q[:, :, None] * r[None, None, :]) / N)
        out[pi] = np.einsum("rc,qrc->q", img, ph)
    del p
    return out


# --------------------------------------------------------------------------
# the grid transform
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [16, 24, 32, 64])
def test_grid_matches_bruteforce_dft(N):
    img = _rng(N).normal(size=(N, N))
    G = oracle.grid(img)
    ref = _brute_grid(img)
    assert np.max(np.abs(G - ref)) <= 1e-13 * np.sum(np.abs(img))


@pytest.mark.parametrize("N", [16, 64, 256])
def test_grid_matches_numpy_rfft2_of_shifted_image(N):
    # Sec. 4: shift -> real-to-complex FFT; rows of G are the unshifted frequencies.
    img = _rng(N + 1).normal(size=(N, N))
    G = oracle.grid(img)
    ref = np.fft.rfft2(np.fft.fftshift(img))
    assert G.shape == ref.shape == (N, N // 2 + 1)
    assert np.max(np.abs(G - ref)) <= 1e-13 * np.sum(np.abs(img))


def test_grid_cell_matches_grid():
    img = _rng(3).normal(size=(32, 32))
    G = oracle.grid(img)
    for p, q in [(0, 0), (5, 3), (31, 16), (16, 0), (17, 11)]:
        assert abs(oracle.grid_cell(img, p, q) - G[p, q]) <= 1e-13 * np.sum(np.abs(img))


@pytest.mark.parametrize("N", [16, 32, 64])
def test_hermitian_columns(N):
    # real image: G[-p, 0] = conj G[p, 0], G[-p, N/2] = conj G[p, N/2]
    img = _rng(N + 7).normal(size=(N, N))
    G = oracle.grid(img)
    p = np.arange(N)
    for q in (0, N // 2):
        assert np.max(np.abs(G[(-p) % N, q] - np.conj(G[p, q]))) <= 1e-13 * np.sum(np.abs(img))


# --------------------------------------------------------------------------
# point sources: constant visibility and the phase ramp (Sec. 3.3)
# --------------------------------------------------------------------------
def test_centred_point_source_is_constant():
    N, dxy, F = 64, 0.02 * ARC, 1.7
    img = np.zeros((N, N))
    img[N // 2, N // 2] = F
    G = oracle.grid(img)
    assert np.max(np.abs(G - F)) <= 1e-15 * F
    du = 1.0 / (N * dxy)
    u, v = wl.uv_uniform_disk(500, 0.9 * (N / 2 - 1) * du, seed=11)
    for PA in (0.0, 0.7, 2.9, -1.3):
        V = oracle.sampleImage(img, dxy, u, v, PA=PA)
        assert np.max(np.abs(V - F)) <= 1e-14 * F
    # with offsets: V = F exp(+2 pi i (u dRA + v dDec)), PA-independent
    dRA, dDec = 0.3 * ARC, -0.17 * ARC
    for PA in (0.0, 1.1):
        V = oracle.sampleImage(img, dxy, u, v, PA=PA, dRA=dRA, dDec=dDec)
        ref = F * np.exp(2j * np.pi * (u * dRA + v * dDec))
        assert np.max(np.abs(V - ref)) <= 1e-14 * F


def test_offcentre_point_source_phase_ramp_at_nodes():
    N, dxy, F = 64, 0.05 * ARC, 0.8
    r0, c0 = 20, 41
    img = np.zeros((N, N))
    img[r0, c0] = F
    x0 = (N // 2 - c0) * dxy
    y0 = (N // 2 - r0) * dxy
    G = oracle.grid(img)
    # closed form on every node: F exp(+2 pi i (q x0 + p~ y0) / (N dxy)), p~ = p - N [p >= N/2]
    p = np.arange(N)[:, None]
    pt = np.where(p >= N // 2, p - N, p)
    q = np.arange(N // 2 + 1)[None, :]
    k = (q * (N // 2 - c0) + pt * (N // 2 - r0)) % N  # exact integer phase index
    ref = F * np.exp(2j * np.pi * k / N)
    assert np.max(np.abs(G - ref)) <= 1e-14 * F
    # sampled exactly on nodes (u = q du, v = p~ du), both half planes (mirrored points too)
    du = 1.0 / (N * dxy)
    rng = _rng(5)
    qq = rng.integers(-(N // 2 - 2), N // 2 - 1, 300).astype(float)
    pp = rng.integers(-(N // 2 - 2), N // 2 - 1, 300).astype(float)
    u, v = qq * du, pp * du
    V = oracle.sampleImage(img, dxy, u, v)
    kk = (qq.astype(int) * (N // 2 - c0) + pp.astype(int) * (N // 2 - r0)) % N
    assert np.max(np.abs(V - F * np.exp(2j * np.pi * kk / N))) <= 1e-13 * F
    # the same visibility through the continuous formula exp(+2 pi i (u x0 + v y0))
    assert np.max(np.abs(V - F * np.exp(2j * np.pi * (u * x0 + v * y0)))) <= 1e-12 * F


def test_rotation_convention_north_to_east():
    # Sec. 2.2 / Sec. 3.3: PA is measured East of North.  A point 6 px North of
    # the centre rotated by PA = 90 deg must look like a point 6 px East.
    N, dxy, F = 64, 0.05 * ARC, 1.0
    north = np.zeros((N, N)); north[N // 2 - 6, N // 2] = F
    east = np.zeros((N, N)); east[N // 2, N // 2 - 6] = F
    du = 1.0 / (N * dxy)
    rng = _rng(9)
    # uv points whose rotated coordinates land on nodes
    qq = rng.integers(-(N // 2 - 3), N // 2 - 2, 200).astype(float)
    pp = rng.integers(-(N // 2 - 3), N // 2 - 2, 200).astype(float)
    PA = math.pi / 2
    # inverse rotation of (q du, p du): u = u' cos + v' sin, v = -u' sin + v' cos
    u = qq * du * math.cos(PA) + pp * du * math.sin(PA)
    v = -qq * du * math.sin(PA) + pp * du * math.cos(PA)
    V_rot = oracle.sampleImage(north, dxy, u, v, PA=PA)
    V_east = oracle.sampleImage(east, dxy, u, v, PA=0.0)
    assert np.max(np.abs(V_rot - V_east)) <= 1e-12 * F
    # and the East source has the positive-x phase ramp: x0 = +6 dxy
    assert np.max(np.abs(V_east - F * np.exp(2j * np.pi * u * 6 * dxy))) <= 1e-12 * F


# --------------------------------------------------------------------------
# Gaussian closed form (the FT of a sampled Gaussian, aliasing negligible)
# --------------------------------------------------------------------------
def test_gaussian_closed_form():
    N, dxy, F = 128, 0.01 * ARC, 1.3
    sx, sy = 4.0 * dxy, 3.0 * dxy          # sigma >= 3 dxy, N dxy / 2 >= 8 sigma
    img = wl.gaussian_image(N, dxy, F, sx, sy)
    du = 1.0 / (N * dxy)
    G = oracle.grid(img)
    p = np.arange(N)[:, None]
    pt = np.where(p >= N // 2, p - N, p)
    q = np.arange(N // 2 + 1)[None, :]
    ref = F * np.exp(-2 * np.pi**2 * ((sx * q * du) ** 2 + (sy * pt * du) ** 2))
    assert np.max(np.abs(G - ref)) <= 1e-12 * F
    # off the nodes the bilinear error is bounded by du^2/8 (max|d2V/du2| + max|d2V/dv2|)
    u, v = wl.uv_uniform_disk(2000, 0.8 * (N / 2 - 1) * du, seed=21)
    PA = 0.4
    V = oracle.sampleImage(img, dxy, u, v, PA=PA)
    ur = u * math.cos(PA) - v * math.sin(PA)
    vr = u * math.sin(PA) + v * math.cos(PA)
    Vref = F * np.exp(-2 * np.pi**2 * ((sx * ur) ** 2 + (sy * vr) ** 2))
    bound = du**2 / 8 * (4 * np.pi**2 * sx**2 * F + 4 * np.pi**2 * sy**2 * F) + 1e-12 * F
    err = np.abs(V - Vref)
    assert np.max(err) <= bound
    assert np.max(np.abs(V.imag)) <= 1e-12 * F      # centred even image: real V


def test_inclination_deprojection_of_image():
    # Reading of the paper's inclination for *Image: the image stretched along x by
    # 1/cos(inc) before rotation.  A circular Gaussian deprojected must match the
    # closed form of the inclined (elliptical) Gaussian cos(i) F exp(-2 pi^2 s^2 ((u' cos i)^2 + v'^2)).
    N, dxy, F = 128, 0.01 * ARC, 1.0
    s = 4.0 * dxy
    img = wl.gaussian_image(N, dxy, F, s, s)
    du = 1.0 / (N * dxy)
    u, v = wl.uv_uniform_disk(1500, 0.8 * (N / 2 - 1) * du, seed=31)
    inc, PA = 50 * wl.DEG, 0.9
    V = oracle.sampleImage(img, dxy, u, v, PA=PA, inc=inc)
    ur = (u * math.cos(PA) - v * math.sin(PA)) * math.cos(inc)
    vr = u * math.sin(PA) + v * math.cos(PA)
    Vref = math.cos(inc) * F * np.exp(-2 * np.pi**2 * s**2 * (ur**2 + vr**2))
    bound = du**2 / 8 * 8 * np.pi**2 * s**2 * F + 1e-12
    assert np.max(np.abs(V - Vref)) <= bound


# --------------------------------------------------------------------------
# bilinear sampling against scipy (Sec. 3.4: 4-node bilinear interpolation)
# --------------------------------------------------------------------------
def test_bilinear_matches_scipy_spline_degree_one():
    N, dxy = 64, 0.02 * ARC
    img = _rng(41).normal(size=(N, N))
    G = oracle.grid(img)
    S = np.fft.fftshift(G, axes=0)   # row i <-> frequency i - N/2 (library shift)
    du = 1.0 / (N * dxy)
    rng = _rng(42)
    u = rng.uniform(0.0, (N / 2 - 1.01) * du, 800)        # u > 0: no mirroring
    v = rng.uniform(-(N / 2 - 1.01) * du, (N / 2 - 1.01) * du, 800)
    V = oracle.sampleImage(img, dxy, u, v)
    rows, cols = np.arange(N, dtype=float), np.arange(N // 2 + 1, dtype=float)
    sre = RectBivariateSpline(rows, cols, S.real, kx=1, ky=1, s=0)
    sim = RectBivariateSpline(rows, cols, S.imag, kx=1, ky=1, s=0)
    fv, fu = N / 2 + v / du, u / du
    ref = sre.ev(fv, fu) + 1j * sim.ev(fv, fu)
    assert np.max(np.abs(V - ref)) <= 1e-12 * np.max(np.abs(S))


def test_hermitian_sampling_and_mirror():
    # a real image has V(-u, -v) = conj V(u, v); the mirror makes it exact
    N, dxy = 64, 0.02 * ARC
    img = _rng(51).normal(size=(N, N))
    du = 1.0 / (N * dxy)
    u, v = wl.uv_uniform_disk(1000, 0.9 * (N / 2 - 1) * du, seed=52)
    kw = dict(PA=0.77, dRA=0.1 * ARC, dDec=-0.2 * ARC)
    V1 = oracle.sampleImage(img, dxy, u, v, **kw)
    V2 = oracle.sampleImage(img, dxy, -u, -v, **kw)
    assert np.max(np.abs(V2 - np.conj(V1))) <= 1e-14 * np.max(np.abs(V1))


def test_off_grid_points_are_nan():
    N, dxy = 32, 0.02 * ARC
    img = _rng(61).normal(size=(N, N))
    du = 1.0 / (N * dxy)
    # valid iff 0 <= floor(|u'|/du) <= N/2 - 1 and 0 <= floor(N/2 + v'/du) <= N - 2
    u = np.array([0.5, N / 2 - 0.5, 0.0, 0.0, (N / 2 + 0.2), 0.0, 3.2]) * du
    v = np.array([0.5, 0.0, N / 2 - 1.5, -(N / 2 - 0.25), 0.0, N / 2 - 0.5, -(N / 2 + 0.3)]) * du
    V = oracle.sampleImage(img, dxy, u, v)
    assert np.all(np.isfinite(V[:4]))
    assert np.all(np.isnan(V[4:]))


def test_sample_direct_matches_sample_grid():
    N, dxy = 48, 0.02 * ARC
    img = _rng(71).normal(size=(N, N))
    du = 1.0 / (N * dxy)
    u, v = wl.uv_uniform_disk(50, 0.9 * (N / 2 - 1) * du, seed=72)
    kw = dict(PA=2.1, dRA=0.05 * ARC, dDec=0.02 * ARC, inc=0.4)
    V1 = oracle.sampleImage(img, dxy, u, v, **kw)
    V2 = oracle.sample_direct(img, dxy, u, v, **kw)
    assert np.max(np.abs(V1 - V2)) <= 1e-13 * np.sum(np.abs(img))


def test_linearity():
    N, dxy = 32, 0.02 * ARC
    rng = _rng(81)
    A, B = rng.normal(size=(N, N)), rng.normal(size=(N, N))
    du = 1.0 / (N * dxy)
    u, v = wl.uv_uniform_disk(300, 0.9 * (N / 2 - 1) * du, seed=82)
    kw = dict(PA=1.0, dRA=0.03 * ARC, dDec=0.0, inc=0.2)
    a, b = 0.7, -2.5
    lhs = oracle.sampleImage(a * A + b * B, dxy, u, v, **kw)
    rhs = a * oracle.sampleImage(A, dxy, u, v, **kw) + b * oracle.sampleImage(B, dxy, u, v, **kw)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.sum(np.abs(A) + np.abs(B))


# --------------------------------------------------------------------------
# the sweep (Sec. 2.2, Sec. 4, App. D)
# --------------------------------------------------------------------------
def test_sweep_reproduces_linear_profile():
    # linear interpolation is exact on a linear profile; outside [Rmin, Rmax] -> 0;
    # the centre pixel is the extrapolation to rho = 0.
    N, dxy = 64, 0.1 * ARC
    Rmin, Nr = 0.35 * dxy, 40
    dR = 0.5 * dxy
    a, b = 3.0, -0.2 / dxy
    r = Rmin + dR * np.arange(Nr)
    I = a + b * r
    inc = 0.5
    img = oracle.sweep(I, Rmin, dR, N, dxy, inc)
    x = (N // 2 - np.arange(N)) * dxy
    X = x[None, :] / math.cos(inc)
    Y = x[:, None]
    rho = np.sqrt(X**2 + Y**2)
    inside = (rho >= Rmin) & (rho <= Rmin + dR * (Nr - 1))
    ref = np.where(inside, (a + b * rho) * dxy**2, 0.0)
    ref[N // 2, N // 2] = a * dxy**2
    assert np.max(np.abs(img - ref)) <= 1e-13 * a * dxy**2
    assert np.count_nonzero(img) == np.count_nonzero(inside) + (0 if inside[N // 2, N // 2] else 1)


def test_sweep_matches_scipy_interp1d():
    N, dxy = 96, 0.03 * ARC
    rng = _rng(91)
    Nr = 57
    Rmin, dR = 0.2 * dxy, 0.7 * dxy
    I = rng.random(Nr) * 1e10
    inc = 0.8
    img = oracle.sweep(I, Rmin, dR, N, dxy, inc)
    x = (N // 2 - np.arange(N)) * dxy
    rho = np.sqrt((x[None, :] / math.cos(inc)) ** 2 + x[:, None] ** 2)
    grid = Rmin + dR * np.arange(Nr)
    f = interp1d(grid, I, kind="linear", bounds_error=False, fill_value=0.0, assume_sorted=True)
    ref = f(rho) * dxy**2
    fc = interp1d(grid, I, kind="linear", bounds_error=False, fill_value="extrapolate",
                  assume_sorted=True)
    ref[N // 2, N // 2] = fc(0.0) * dxy**2
    assert np.max(np.abs(img - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_sweep_symmetry_and_profile_visibilities_are_real():
    # a swept image is symmetric under x -> -x and y -> -y (columns c <-> N - c,
    # rows r <-> N - r for c, r >= 1), so V is real at zero offsets for any PA
    # (Sec. 5: the imaginary part vanishes for axisymmetric images).
    case = wl.random_case(64, 400, seed=101, kind="profile")
    img = oracle.sweep(case.I, case.Rmin, case.dR, case.N, case.dxy, case.inc)
    N = case.N
    assert np.array_equal(img[1:, 1:], img[1:, 1:][::-1, :])
    assert np.array_equal(img[1:, 1:], img[1:, 1:][:, ::-1])
    # keep the support inside the symmetric part: zero the first row / column
    img2 = img.copy(); img2[0, :] = 0.0; img2[:, 0] = 0.0
    V = oracle.sampleImage(img2, case.dxy, case.u, case.v, PA=case.PA)
    assert np.max(np.abs(V.imag)) <= 1e-14 * np.max(np.abs(V))
    del N


def test_swept_profile_visibilities_are_even_in_u_and_v():
    # the swept disc before rotation is symmetric about both axes, so its grid
    # spectrum is real and even in u and in v separately, and so is the
    # bilinear interpolant of it (Sec. 3.4; App. D's mirror included): at
    # PA = 0 and zero offsets V(u, v) = V(-u, v) = V(u, -v) = V(-u, -v), also
    # between nodes and across the v = 0 line.  A mirror that reads the wrong
    # node, or a row index off by one (0.8 of max|V| for one row), breaks it.
    case = wl.random_case(64, 10, seed=121, kind="profile")
    N, dxy = case.N, case.dxy
    du = 1.0 / (N * dxy)
    rng = np.random.default_rng(5)
    u = np.concatenate([rng.uniform(0.0, N / 2 - 1.5, 300), [0.3, 2.7, 0.0]]) * du
    v = np.concatenate([rng.uniform(-(N / 2 - 1.5), N / 2 - 1.5, 300), [-0.3, 0.4, -3.5]]) * du

    def V(uu, vv):
        return oracle.sampleProfile(case.I, case.Rmin, case.dR, N, dxy, uu, vv, inc=case.inc)

    V0 = V(u, v)
    scale = np.max(np.abs(V0))
    for W in (V(-u, v), V(u, -v), V(-u, -v)):
        assert np.max(np.abs(W - V0)) <= 1e-13 * scale
    assert np.max(np.abs(V0.imag)) <= 1e-14 * scale


def test_profile_path_is_image_path_of_sweep():
    case = wl.random_case(64, 300, seed=111, kind="profile")
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec)
    V1 = oracle.sampleProfile(case.I, case.Rmin, case.dR, case.N, case.dxy, case.u, case.v,
                              inc=case.inc, **kw)
    img = oracle.sweep(case.I, case.Rmin, case.dR, case.N, case.dxy, case.inc)
    V2 = oracle.sampleImage(img, case.dxy, case.u, case.v, **kw)
    assert np.array_equal(V1, V2)


# --------------------------------------------------------------------------
# chi-square (Sec. 3.1, Eq. def.chi.square)
# --------------------------------------------------------------------------
def test_chi2_zero_at_model_and_noise_sum():
    case = wl.random_case(32, 5000, seed=121)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=case.inc)
    V = oracle.sampleImage(case.image, case.dxy, case.u, case.v, **kw)
    assert oracle.chi2Image(case.image, case.dxy, case.u, case.v, V.real, V.imag, case.w,
                            **kw) == 0.0
    re, im = V.real + case.noise_re, V.imag + case.noise_im
    c2 = oracle.chi2Image(case.image, case.dxy, case.u, case.v, re, im, case.w, **kw)
    # the residual is exactly the noise up to the rounding of V + n - V
    dre = (V.real + case.noise_re) - V.real
    dim = (V.imag + case.noise_im) - V.imag
    ref = math.fsum(case.w * (dre**2 + dim**2))
    assert abs(c2 - ref) <= 1e-13 * ref
    # and it is chi-square distributed with 2M degrees of freedom (w ~ 1/sigma^2 up to the scale)
    c2n = math.fsum((case.noise_re**2 + case.noise_im**2) / 1e-6)
    assert abs(c2n - 2 * case.M) < 6 * math.sqrt(4 * case.M)


# --------------------------------------------------------------------------
# gradients: exact transpose (chi^2 is quadratic in the pixels / profile values)
# --------------------------------------------------------------------------
def test_grad_image_matches_linearity_definition():
    case = wl.random_case(8, 40, seed=131)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=case.inc)
    re = case.noise_re + 0.3
    im = case.noise_im - 0.1
    c2, g = oracle.grad_image(case.image, case.dxy, case.u, case.v, re, im, case.w, **kw)
    V = oracle.sampleImage(case.image, case.dxy, case.u, case.v, **kw)
    R = (re + 1j * im) - V
    N = case.N
    ref = np.empty((N, N))
    for r in range(N):
        for c in range(N):
            e = np.zeros((N, N)); e[r, c] = 1.0
            Ve = oracle.sampleImage(e, case.dxy, case.u, case.v, **kw)
            ref[r, c] = -2.0 * np.sum(case.w * np.real(np.conj(R) * Ve))
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_grad_image_central_differences_are_exact():
    case = wl.random_case(16, 200, seed=141)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=case.inc)
    re, im = case.noise_re + 0.2, case.noise_im
    _, g = oracle.grad_image(case.image, case.dxy, case.u, case.v, re, im, case.w, **kw)
    rng = _rng(142)
    h = 0.5
    for _ in range(12):
        r, c = rng.integers(0, case.N, 2)
        ip = case.image.copy(); ip[r, c] += h
        im_ = case.image.copy(); im_[r, c] -= h
        fd = (oracle.chi2Image(ip, case.dxy, case.u, case.v, re, im, case.w, **kw)
              - oracle.chi2Image(im_, case.dxy, case.u, case.v, re, im, case.w, **kw)) / (2 * h)
        assert abs(fd - g[r, c]) <= 1e-7 * (abs(g[r, c]) + 1e-3 * np.max(np.abs(g)))


def test_grad_profile_central_differences_are_exact():
    case = wl.random_case(32, 300, seed=151, kind="profile", Nr=24)
    kw = dict(inc=case.inc, PA=case.PA, dRA=case.dRA, dDec=case.dDec)
    args = (case.Rmin, case.dR, case.N, case.dxy, case.u, case.v)
    re, im = case.noise_re + 0.2, case.noise_im
    _, gI = oracle.grad_profile(case.I, *args, re, im, case.w, **kw)
    h = 0.25 * np.max(np.abs(case.I))
    for j in [0, 1, 2, 7, 15, 23]:
        Ip = case.I.copy(); Ip[j] += h
        Im = case.I.copy(); Im[j] -= h
        fd = (oracle.chi2Profile(Ip, *args, re, im, case.w, **kw)
              - oracle.chi2Profile(Im, *args, re, im, case.w, **kw)) / (2 * h)
        assert abs(fd - gI[j]) <= 1e-7 * (abs(gI[j]) + 1e-3 * np.max(np.abs(gI)))


def test_grad_adjoint_dot_product():
    # <d chi2 / d img, delta> equals the directional derivative for any delta
    case = wl.random_case(24, 400, seed=161)
    kw = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=case.inc)
    re, im = case.noise_re + 0.1, case.noise_im + 0.05
    _, g = oracle.grad_image(case.image, case.dxy, case.u, case.v, re, im, case.w, **kw)
    d = _rng(162).normal(size=g.shape)
    h = 0.1
    fp = oracle.chi2Image(case.image + h * d, case.dxy, case.u, case.v, re, im, case.w, **kw)
    fm = oracle.chi2Image(case.image - h * d, case.dxy, case.u, case.v, re, im, case.w, **kw)
    assert abs((fp - fm) / (2 * h) - np.sum(g * d)) <= 1e-8 * abs(np.sum(np.abs(g * d)))


# ---- geometry gradients (not in the paper) --------------------------------
def _geo_obs(rng, M, scale):
    return (rng.normal(0, scale, M), rng.normal(0, scale, M), rng.uniform(0.5, 2.0, M))


def test_geograd_point_source_closed_form():
    # a centred point source has G = F at every node: V = cos(inc) F exp(i theta),
    # so the offset and inclination derivatives are explicit and d/dPA = 0
    N, dxy, F = 32, 1e-7, 1.7
    img = np.zeros((N, N))
    img[N // 2, N // 2] = F
    rng = np.random.default_rng(31)
    M = 400
    du = 1.0 / (N * dxy)
    rho = du * 10 * np.sqrt(rng.uniform(0, 1, M))
    phi = rng.uniform(0, 2 * np.pi, M)
    u, v = rho * np.cos(phi), rho * np.sin(phi)
    re, im, w = _geo_obs(rng, M, 1.0)
    PA, dRA, dDec, inc = 0.7, 3e-7, -2e-7, 0.4
    c2, g = oracle.geograd_image(img, dxy, u, v, re, im, w, PA, dRA, dDec, inc)
    theta = 2 * np.pi * (u * dRA + v * dDec)
    V = np.cos(inc) * F * np.exp(1j * theta)
    R = re + 1j * im - V
    d_dRA = np.sum(-2 * w * np.real(np.conj(R) * 2j * np.pi * u * V))
    d_dDec = np.sum(-2 * w * np.real(np.conj(R) * 2j * np.pi * v * V))
    d_inc = np.sum(-2 * w * np.real(np.conj(R) * (-np.sin(inc)) * F * np.exp(1j * theta)))
    assert abs(c2 - np.sum(w * np.abs(R) ** 2)) <= 1e-12 * c2
    assert abs(g[0]) <= 1e-12 * np.sum(w * np.abs(R) * F)
    for got, want in ((g[1], d_dRA), (g[2], d_dDec), (g[3], d_inc)):
        assert abs(got - want) <= 1e-10 * abs(want), (got, want)


def _central(f, x0, h):
    return (f(x0 + h) - f(x0 - h)) / (2 * h)


@pytest.mark.parametrize("kind", ["image", "profile"])
def test_geograd_matches_central_differences(kind):
    # the derivative formulas against the derivative of the (separately pinned)
    # forward chi^2; steps small enough that no point crosses a cell edge
    case = wl.random_case(32, 600, seed=3300 + (kind == "profile"), kind=kind, Nr=40, fill=0.7)
    rng = np.random.default_rng(3310)
    re, im, w = _geo_obs(rng, case.M, 0.02)
    base = dict(PA=case.PA, dRA=case.dRA, dDec=case.dDec, inc=0.35)
    if kind == "image":
        f = lambda **kw: oracle.chi2Image(case.image, case.dxy, case.u, case.v, re, im, w, **kw)
        c2, g = oracle.geograd_image(case.image, case.dxy, case.u, case.v, re, im, w, **base)
    else:
        f = lambda **kw: oracle.chi2Profile(case.I, case.Rmin, case.dR, case.N, case.dxy, case.u,
                                            case.v, re, im, w, **kw)
        c2, g = oracle.geograd_profile(case.I, case.Rmin, case.dR, case.N, case.dxy, case.u,
                                       case.v, re, im, w, **base)
    assert abs(c2 - f(**base)) <= 1e-12 * c2
    steps = {"PA": 1e-6, "dRA": 1e-3 * case.dxy, "dDec": 1e-3 * case.dxy, "inc": 1e-6}
    for k, name in enumerate(("PA", "dRA", "dDec", "inc")):
        def fk(x, name=name):
            kw = dict(base)
            kw[name] = x
            return f(**kw)
        fd = _central(fk, base[name], steps[name])
        assert abs(g[k] - fd) <= 1e-5 * max(abs(fd), 1e-3 * c2), (name, g[k], fd)


# ---- several sources (Sec. 3.2) ---------------------------------------------
def test_sources_sum_is_the_transform_of_the_summed_image():
    # sampling is linear in the image: two sources with the same grid and
    # geometry give the visibilities of their summed image
    a = wl.random_case(32, 400, seed=3400)
    b = wl.random_case(32, 400, seed=3401)
    geo = dict(PA=a.PA, dRA=a.dRA, dDec=a.dDec, inc=0.3)
    src = [dict(kind="image", image=a.image, dxy=a.dxy, **geo),
           dict(kind="image", image=b.image, dxy=a.dxy, **geo)]
    Vs = oracle.sample_sources(src, a.u, a.v)
    Vsum = oracle.sampleImage(a.image + b.image, a.dxy, a.u, a.v, **geo)
    assert np.max(np.abs(Vs - Vsum)) <= 1e-12 * np.max(np.abs(Vsum))
    # a point source moved by (dRA, dDec) is the centred one times its phase ramp
    N = 32
    delta = np.zeros((N, N))
    delta[N // 2, N // 2] = 1.0
    V1 = oracle.sample_sources([dict(kind="image", image=delta, dxy=a.dxy, PA=0.0, dRA=2e-7,
                                     dDec=-1e-7, inc=0.0)], a.u, a.v)
    assert np.allclose(V1, np.exp(2j * np.pi * (a.u * 2e-7 - a.v * 1e-7)), rtol=0, atol=1e-13)


def test_sources_sharing_spells_out_the_owner():
    # a source that shares its owner's spectrum with the owner's geometry
    # doubles the owner (image: any inc; profile: the owner's inc applies)
    a = wl.random_case(32, 300, seed=3410)
    img = dict(kind="image", image=a.image, dxy=a.dxy, PA=0.4, dRA=a.dRA, dDec=a.dDec, inc=0.5)
    V = oracle.sample_sources([img, dict(img, image=None, share=0)], a.u, a.v)
    V2 = oracle.sampleImage(2.0 * a.image, a.dxy, a.u, a.v, 0.4, a.dRA, a.dDec, 0.5)
    assert np.max(np.abs(V - V2)) <= 1e-12 * np.max(np.abs(V2))
    p = wl.random_case(32, 300, seed=3411, kind="profile")
    prof = dict(kind="profile", I=p.I, Rmin=p.Rmin, dR=p.dR, Nxy=p.N, dxy=p.dxy, inc=0.6, PA=0.2,
                dRA=0.0, dDec=0.0)
    # the sharer's own inc is not used: the transform is the owner's
    sharer = dict(kind="profile", I=None, Rmin=None, dR=None, Nxy=None, dxy=None, inc=1.2, PA=0.2,
                  dRA=3 * p.dxy, dDec=0.0, share=0)
    V = oracle.sample_sources([prof, sharer], p.u, p.v)
    V0 = oracle.sampleProfile(p.I, p.Rmin, p.dR, p.N, p.dxy, p.u, p.v, 0.6, 0.2, 0.0, 0.0)
    ramp = np.exp(2j * np.pi * p.u * 3 * p.dxy)
    assert np.max(np.abs(V - V0 * (1.0 + ramp))) <= 1e-12 * np.max(np.abs(V0))


def test_grad_sources_matches_central_differences():
    # a scene of an image, a profile and a copy of the profile elsewhere:
    # every gradient entry (the owner's including its copy) against central
    # differences of chi2_sources
    a = wl.random_case(16, 120, seed=3420)
    p = wl.random_case(16, 120, seed=3421, kind="profile", Nr=10)
    p.I[:] = p.I / np.max(p.I) * np.max(np.abs(a.image)) / p.dxy ** 2 * 0.3
    src = [dict(kind="image", image=a.image, dxy=a.dxy, PA=0.3, dRA=a.dRA, dDec=a.dDec, inc=0.4),
           dict(kind="profile", I=p.I, Rmin=p.Rmin, dR=p.dR, Nxy=16, dxy=a.dxy, inc=0.5, PA=1.0,
                dRA=0.0, dDec=0.0),
           dict(kind="profile", I=None, PA=2.0, dRA=2 * a.dxy, dDec=-a.dxy, share=1)]
    V = oracle.sample_sources(src, a.u, a.v)
    re, im = 1.1 * V.real + a.noise_re, 0.9 * V.imag + a.noise_im
    c2, g = oracle.grad_sources(src, a.u, a.v, re, im, a.w)
    assert g[2] is None and g[0].shape == a.image.shape and g[1].shape == p.I.shape
    assert abs(c2 - oracle.chi2_sources(src, a.u, a.v, re, im, a.w)) <= 1e-13 * c2

    def f_img(k, h):
        x = a.image.copy()
        x.flat[k] += h
        s = [dict(src[0], image=x), src[1], src[2]]
        return oracle.chi2_sources(s, a.u, a.v, re, im, a.w)

    def f_prof(k, h):
        x = p.I.copy()
        x[k] += h
        s = [src[0], dict(src[1], I=x), src[2]]
        return oracle.chi2_sources(s, a.u, a.v, re, im, a.w)

    rng = np.random.default_rng(3422)
    hi = 1e-4 * np.max(np.abs(a.image))
    for k in rng.choice(a.image.size, 12, replace=False):
        fd = (f_img(k, hi) - f_img(k, -hi)) / (2 * hi)
        assert abs(g[0].flat[k] - fd) <= 1e-6 * np.max(np.abs(g[0])), (k, g[0].flat[k], fd)
    hp = 1e-4 * np.max(p.I)
    for k in range(p.I.size):
        fd = (f_prof(k, hp) - f_prof(k, -hp)) / (2 * hp)
        assert abs(g[1][k] - fd) <= 1e-6 * np.max(np.abs(g[1])), (k, g[1][k], fd)


# ---- image size criteria (Sec. 3.4) -----------------------------------------
def _matrix_table():
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "matrix_sizes_table.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append((f[0] + " " + f[1], float(f[2]), float(f[3]), int(f[4]), float(f[6]),
                     float(f[7]), float(f[8])))
    return rows


def test_image_size_reproduces_the_paper_table():
    # every row of the paper's table: N (iia) exactly, the pixel size and the
    # resolution to the printed digits (f_min = 5, f_max = 2.5, Gamma = 0.6)
    rows = _matrix_table()
    assert len(rows) == 14
    arcsec = np.pi / 648000.0
    for name, bmin, bmax, N_iia, dth, res, lam in rows:
        # two points on the extreme baselines, along different directions
        u = np.array([bmin / lam, 0.0])
        v = np.array([0.0, bmax / lam])
        N, dxy = oracle.get_image_size(u, v)
        assert N == N_iia, (name, N, N_iia)
        assert abs(dxy / arcsec - dth) <= 0.5e-3 + 1e-12, (name, dxy / arcsec, dth)
        assert abs(lam / bmax / arcsec - res) <= 0.5e-3 + 1e-12, name


def test_image_size_primary_beam_criterion():
    # (iib): the image spans the beam exactly and the grid is the smallest
    # power of two reaching f_max rho_max
    rng = np.random.default_rng(3500)
    for _ in range(20):
        r = np.exp(rng.uniform(np.log(1e4), np.log(1e7), 50))
        a = rng.uniform(0, 2 * np.pi, 50)
        u, v = r * np.cos(a), r * np.sin(a)
        PB = rng.uniform(5.0, 60.0) * np.pi / 648000.0
        N, dxy = oracle.get_image_size(u, v, PB=PB)
        assert abs(N * dxy - PB) <= 1e-15 * PB
        du = 1.0 / PB
        assert N * du / 2 >= 2.5 * r.max() > (N // 2) * du / 2


def test_image_size_smooth_hand_worked():
    # with PB = 1 the uv cell is 1 and criterion (i) reads N >= 2 f_max rho_max;
    # the smallest even 2^a 3^b 5^c at or above the bound, worked by hand:
    # 47 -> 48 = 2^4 3, 98 -> 100 = 2^2 5^2, 61 -> 64 = 2^6, 121 -> 128
    # (122 = 2 61, 124 = 4 31, 126 = 2 3^2 7), 17 -> 18 = 2 3^2
    for bound, N_expect in ((47, 48), (98, 100), (61, 64), (121, 128), (17, 18)):
        rho = (bound - 0.5) / 5.0   # 2 f_max rho = bound - 0.5 with f_max = 2.5
        u, v = np.array([rho, 0.3 * rho]), np.array([0.0, 0.1 * rho])
        N, dxy = oracle.get_image_size(u, v, PB=1.0, smooth=True)
        assert N == N_expect, (bound, N)
        assert dxy == 1.0 / N_expect
        # the power-of-two rule on the same points
        N2, _ = oracle.get_image_size(u, v, PB=1.0)
        assert N2 == 1 << (N_expect - 1).bit_length()
