/*
 * oracle.c -- plain FP64 CPU reference of the visibility / chi-square path of
 * Tazzari, Beaujean & Testi, "GALARIO: a GPU accelerated library for
 * analysing radio interferometer observations" (MNRAS 2018, arXiv:1709.06999).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the HIP
 * library.  It shares no code, header, table or constant with it; only the
 * test suite, the smoke entry and the CPU-baseline leg of the benchmark may
 * load it.  Nothing here is tuned: every step is written the slow, obvious way
 * so that it can be compared with the paper by eye.
 *
 * Conventions (the paper's Appendix D reference functions; the body text in
 * Sec. 3.1 writes the conjugate convention -- see the header of oracle/__init__.py):
 *   - image img[r*N + c], r = row (North at r = 0), c = column (East at c = 0),
 *     pixel centre x_c = (N/2 - c) dxy, y_r = (N/2 - r) dxy (Sec. 2.2, App. D);
 *   - the Fourier transform of the image with its origin moved to pixel
 *     (N/2, N/2) is the half spectrum
 *        G[p][q] = sum_{r,c} img[r][c] exp(-2 pi i (p (r - N/2) + q (c - N/2)) / N)
 *     for p in [0, N), q in [0, N/2]  (Sec. 4: shift -> real-to-complex FFT ->
 *     shift), which equals sum img exp(+2 pi i (u x + v y)) at u = q du,
 *     v = p~ du, p~ = p - N [p >= N/2], du = 1 / (N dxy)  (Sec. 3.4);
 *   - complex arrays are interleaved (re, im) doubles.
 *
 * Parity of every function below is pinned in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559
#define TWO_PI_L 6.283185307179586476925286766559L

/* Threads for the following calls (n < 1: all cores).  Timing only: the
 * results do not depend on it. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n >= 1 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* W[m] = exp(-2 pi i m / N), m in [0, N).  Only the oracle uses this table. */
static void orc_twiddles(int64_t N, double *wr, double *wi)
{
    for (int64_t m = 0; m < N; ++m) {
        long double a = TWO_PI_L * (long double)m / (long double)N;
        wr[m] = (double)cosl(a);
        wi[m] = (double)(-sinl(a));
    }
}

/* ------------------------------------------------------------------------ */
/* Sweep: axisymmetric, optionally inclined image from a radial profile.
 * Sec. 2.2 (sampleProfile, inc), Sec. 4 ("Create image"), App. D
 * (py_chi2Profile).  Readings:
 *   - radial grid r_j = Rmin + j dR, j = 0..Nr-1, linear interpolation in
 *     radius, 0 outside the closed interval [Rmin, Rmin + (Nr-1) dR];
 *   - the inclination stretches x: rho = sqrt((x / cos inc)^2 + y^2), a tilt
 *     about the North-South axis (Fig. conventions in Sec. 2.2);
 *   - the centre pixel (N/2, N/2) takes the straight line through (r_0, I_0),
 *     (r_1, I_1) evaluated at rho = 0;
 *   - every value is multiplied by dxy^2 (Jy/sr -> Jy/pixel).
 * Returns 0 on success, -2 on bad sizes, -4 on bad scalars. */
int orc_sweep(const double *I, int64_t Nr, double Rmin, double dR, int64_t N,
              double dxy, double inc, double *img)
{
    if (Nr < 2 || N < 2 || (N % 2) != 0) return -2;
    if (!(dR > 0.0) || !(dxy > 0.0) || !(cos(inc) > 0.0) || !(Rmin >= 0.0)) return -4;
    const double cos_inc = cos(inc);
    const double pix_area = dxy * dxy;
    const double t_max = (double)(Nr - 1);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        const double y = (double)(N / 2 - r) * dxy;
        for (int64_t c = 0; c < N; ++c) {
            const double x = (double)(N / 2 - c) * dxy;
            const double xs = x / cos_inc;
            const double rho = sqrt(xs * xs + y * y);
            const double t = (rho - Rmin) / dR;
            double val;
            if (t >= 0.0 && t <= t_max) {
                int64_t j = (int64_t)floor(t);
                if (j > Nr - 2) j = Nr - 2;
                const double f = t - (double)j;
                val = (1.0 - f) * I[j] + f * I[j + 1];
            } else {
                val = 0.0;
            }
            img[r * N + c] = val * pix_area;
        }
    }
    /* centre pixel: extrapolation of the first segment to rho = 0 */
    const double centre = I[0] - Rmin * (I[1] - I[0]) / dR;
    img[(N / 2) * N + (N / 2)] = centre * pix_area;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Half spectrum by direct (slow) DFT, computed separably: first along each
 * row (c -> q), then along each column (r -> p).  Both sums run over the
 * exact integer phase index (k * n) mod N into the twiddle table, with the
 * origin at pixel N/2 (Sec. 4: the shift before and after the transform).
 * G is [N][N/2+1] interleaved complex.  Cost ~ N^3. */
int orc_grid(const double *img, int64_t N, double *G)
{
    if (N < 2 || (N % 2) != 0) return -2;
    const int64_t NQ = N / 2 + 1;
    double *wr = (double *)malloc(sizeof(double) * N);
    double *wi = (double *)malloc(sizeof(double) * N);
    double *rowre = (double *)malloc(sizeof(double) * N * NQ);
    double *rowim = (double *)malloc(sizeof(double) * N * NQ);
    if (!wr || !wi || !rowre || !rowim) {
        free(wr); free(wi); free(rowre); free(rowim);
        return -5;
    }
    orc_twiddles(N, wr, wi);

    /* row sums: H[r][q] = sum_c img[r][c] W^{q (c - N/2)} */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        for (int64_t q = 0; q < NQ; ++q) {
            double sre = 0.0, sim = 0.0;
            for (int64_t c = 0; c < N; ++c) {
                int64_t k = (q * (c - N / 2)) % N;
                if (k < 0) k += N;
                sre += img[r * N + c] * wr[k];
                sim += img[r * N + c] * wi[k];
            }
            rowre[r * NQ + q] = sre;
            rowim[r * NQ + q] = sim;
        }
    }
    /* column sums: G[p][q] = sum_r H[r][q] W^{p (r - N/2)} */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        for (int64_t q = 0; q < NQ; ++q) {
            double sre = 0.0, sim = 0.0;
            for (int64_t r = 0; r < N; ++r) {
                int64_t k = (p * (r - N / 2)) % N;
                if (k < 0) k += N;
                const double hr = rowre[r * NQ + q], hi = rowim[r * NQ + q];
                sre += hr * wr[k] - hi * wi[k];
                sim += hr * wi[k] + hi * wr[k];
            }
            G[2 * (p * NQ + q)] = sre;
            G[2 * (p * NQ + q) + 1] = sim;
        }
    }
    free(wr); free(wi); free(rowre); free(rowim);
    return 0;
}

/* One cell G[p][q] by the non-separable double sum over all pixels, the
 * phase index p (r - N/2) + q (c - N/2) reduced mod N exactly. */
void orc_grid_cell(const double *img, int64_t N, int64_t p, int64_t q, double *out2)
{
    double *wr = (double *)malloc(sizeof(double) * N);
    double *wi = (double *)malloc(sizeof(double) * N);
    orc_twiddles(N, wr, wi);
    double sre = 0.0, sim = 0.0;
    for (int64_t r = 0; r < N; ++r) {
        for (int64_t c = 0; c < N; ++c) {
            int64_t k = (p * (r - N / 2) + q * (c - N / 2)) % N;
            if (k < 0) k += N;
            sre += img[r * N + c] * wr[k];
            sim += img[r * N + c] * wi[k];
        }
    }
    free(wr);
    free(wi);
    out2[0] = sre;
    out2[1] = sim;
}

/* ------------------------------------------------------------------------ */
/* Where one (u, v) point falls on the shifted half spectrum.
 * Sec. 3.3: rotate the uv point by PA (u' = u cosPA - v sinPA,
 * v' = u sinPA + v cosPA).  Extension (documented reading): a non-zero inc
 * deprojects u' <- u' cos(inc) and scales the flux by cos(inc).
 * App. D / Sec. 3.4: points with u' < 0 are mirrored to (-u', -v') and the
 * sample is conjugated (the real-to-complex transform only stores u >= 0);
 * fractional indices fu = u'/du, fv = N/2 + v'/du on the grid whose row i
 * holds frequency p~ = i - N/2.  A point is valid only when all four nodes
 * of its bilinear stencil exist: 0 <= floor(fu) <= N/2 - 1 and
 * 0 <= floor(fv) <= N - 2.
 * Returns 1 if valid, 0 otherwise. */
typedef struct {
    int64_t i0, j0;   /* shifted row, column of the lower-left node */
    double s, t;      /* fractional offsets along u and v */
    int conj;         /* 1 if the point was mirrored */
} orc_stencil;

static int orc_locate(double u, double v, int64_t N, double du, double cpa,
                      double spa, double cinc, orc_stencil *st)
{
    double ur = u * cpa - v * spa;
    double vr = u * spa + v * cpa;
    ur = ur * cinc;
    st->conj = 0;
    if (ur < 0.0) {
        ur = -ur;
        vr = -vr;
        st->conj = 1;
    }
    const double fu = ur / du;
    const double fv = (double)(N / 2) + vr / du;
    const double j0f = floor(fu), i0f = floor(fv);
    if (!(j0f >= 0.0 && j0f <= (double)(N / 2 - 1))) return 0;
    if (!(i0f >= 0.0 && i0f <= (double)(N - 2))) return 0;
    st->j0 = (int64_t)j0f;
    st->i0 = (int64_t)i0f;
    st->s = fu - j0f;
    st->t = fv - i0f;
    return 1;
}

/* Value of the shifted spectrum S[i][q] = G[(i - N/2) mod N][q]. */
static void orc_shifted(const double *G, int64_t N, int64_t i, int64_t q, double *re, double *im)
{
    const int64_t NQ = N / 2 + 1;
    int64_t p = (i - N / 2) % N;
    if (p < 0) p += N;
    *re = G[2 * (p * NQ + q)];
    *im = G[2 * (p * NQ + q) + 1];
}

/* Bilinear interpolation on the four nodes (Sec. 3.4, Press et al.), the
 * conjugation of mirrored points, the inclination flux factor, and the
 * translation by the phase exp(+i theta), theta = 2 pi (u dRA + v dDec)
 * with the sky (unrotated) uv and offsets (Sec. 3.3, App. D). */
static void orc_finish(double b00r, double b00i, double b01r, double b01i,
                       double b10r, double b10i, double b11r, double b11i,
                       const orc_stencil *st, double cinc, double u, double v,
                       double dRA, double dDec, double *out2)
{
    const double s = st->s, t = st->t;
    const double w00 = (1.0 - t) * (1.0 - s), w01 = (1.0 - t) * s;
    const double w10 = t * (1.0 - s), w11 = t * s;
    double br = w00 * b00r + w01 * b01r + w10 * b10r + w11 * b11r;
    double bi = w00 * b00i + w01 * b01i + w10 * b10i + w11 * b11i;
    if (st->conj) bi = -bi;
    br *= cinc;
    bi *= cinc;
    const double theta = TWO_PI * (u * dRA + v * dDec);
    const double c = cos(theta), sn = sin(theta);
    out2[0] = br * c - bi * sn;
    out2[1] = br * sn + bi * c;
}

/* sample the half spectrum G at M uv points; invalid points give NaN.
 * Returns the number of invalid points. */
int64_t orc_sample(const double *G, int64_t N, double dxy, const double *u,
                   const double *v, int64_t M, double PA, double dRA,
                   double dDec, double inc, double *vis)
{
    const double du = 1.0 / ((double)N * dxy);
    const double cpa = cos(PA), spa = sin(PA), cinc = cos(inc);
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t k = 0; k < M; ++k) {
        orc_stencil st;
        if (!orc_locate(u[k], v[k], N, du, cpa, spa, cinc, &st)) {
            vis[2 * k] = NAN;
            vis[2 * k + 1] = NAN;
            bad += 1;
            continue;
        }
        double a[8];
        orc_shifted(G, N, st.i0, st.j0, &a[0], &a[1]);
        orc_shifted(G, N, st.i0, st.j0 + 1, &a[2], &a[3]);
        orc_shifted(G, N, st.i0 + 1, st.j0, &a[4], &a[5]);
        orc_shifted(G, N, st.i0 + 1, st.j0 + 1, &a[6], &a[7]);
        orc_finish(a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], &st, cinc,
                   u[k], v[k], dRA, dDec, &vis[2 * k]);
    }
    return bad;
}

/* Same as orc_sample but each needed node is computed by the non-separable
 * double sum from the image: usable at full image size for a few points. */
int64_t orc_sample_direct(const double *img, int64_t N, double dxy, const double *u,
                          const double *v, int64_t M, double PA, double dRA,
                          double dDec, double inc, double *vis)
{
    const double du = 1.0 / ((double)N * dxy);
    const double cpa = cos(PA), spa = sin(PA), cinc = cos(inc);
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int64_t k = 0; k < M; ++k) {
        orc_stencil st;
        if (!orc_locate(u[k], v[k], N, du, cpa, spa, cinc, &st)) {
            vis[2 * k] = NAN;
            vis[2 * k + 1] = NAN;
            bad += 1;
            continue;
        }
        double a[8];
        for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj) {
                int64_t p = (st.i0 + di - N / 2) % N;
                if (p < 0) p += N;
                orc_grid_cell(img, N, p, st.j0 + dj, &a[2 * (2 * di + dj)]);
            }
        orc_finish(a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], &st, cinc,
                   u[k], v[k], dRA, dDec, &vis[2 * k]);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* chi^2 = sum_k w_k |Vobs_k - Vmod_k|^2  (Sec. 3.1, Eq. def.chi.square), with
 * Neumaier-compensated summation in a fixed serial order. */
double orc_chi2(const double *vis, const double *re, const double *im,
                const double *w, int64_t M)
{
    double sum = 0.0, comp = 0.0;
    for (int64_t k = 0; k < M; ++k) {
        const double dr = vis[2 * k] - re[k];
        const double di = vis[2 * k + 1] - im[k];
        const double term = w[k] * (dr * dr + di * di);
        const double t = sum + term;
        if (fabs(sum) >= fabs(term))
            comp += (sum - t) + term;
        else
            comp += (term - t) + sum;
        sum = t;
    }
    return sum + comp;
}

/* ------------------------------------------------------------------------ */
/* Gradient of chi^2 with respect to the image pixels.  The paper does not
 * differentiate; this is the exact transpose of the linear map
 * img -> V above.  Each sample is V_k = sum_x A_k[x] img[x]; with the
 * residual R_k = Vobs_k - V_k,
 *    d chi^2 / d img[x] = -2 sum_k w_k Re(conj(R_k) A_k[x]).
 * Written out through the steps: every point scatters
 *    a_k = conj(R_k) e^{+i theta_k}      (not mirrored)
 *    a_k = R_k e^{-i theta_k}            (mirrored, u' < 0)
 * times w_k cos(inc) times its bilinear weight onto its four nodes of the
 * half spectrum A[p][q], and the pixel gradient is
 *    g[r][c] = -2 Re sum_{p,q} A[p][q] exp(-2 pi i (p (r-N/2) + q (c-N/2)) / N)
 * summed over the stored nodes only (p in [0,N), q in [0,N/2]), done
 * separably by direct sums.  vis holds the model V_k (from orc_sample).
 * Returns the number of invalid points (their terms are skipped). */
int64_t orc_grad_image(const double *vis, int64_t N, double dxy, const double *u,
                       const double *v, const double *re, const double *im,
                       const double *w, int64_t M, double PA, double dRA,
                       double dDec, double inc, double *grad)
{
    const int64_t NQ = N / 2 + 1;
    const double du = 1.0 / ((double)N * dxy);
    const double cpa = cos(PA), spa = sin(PA), cinc = cos(inc);
    double *Are = (double *)calloc((size_t)(N * NQ), sizeof(double));
    double *Aim = (double *)calloc((size_t)(N * NQ), sizeof(double));
    double *Hre = (double *)calloc((size_t)(N * NQ), sizeof(double));
    double *Him = (double *)calloc((size_t)(N * NQ), sizeof(double));
    double *wr = (double *)malloc(sizeof(double) * N);
    double *wi = (double *)malloc(sizeof(double) * N);
    orc_twiddles(N, wr, wi);
    int64_t bad = 0;
    /* scatter, serial so that the sum order is fixed */
    for (int64_t k = 0; k < M; ++k) {
        orc_stencil st;
        if (!orc_locate(u[k], v[k], N, du, cpa, spa, cinc, &st)) {
            bad += 1;
            continue;
        }
        const double rr = re[k] - vis[2 * k], ri = im[k] - vis[2 * k + 1];
        const double theta = TWO_PI * (u[k] * dRA + v[k] * dDec);
        const double c = cos(theta), sn = sin(theta);
        double ar, ai;
        if (!st.conj) { /* conj(R) e^{i theta} */
            ar = rr * c + ri * sn;
            ai = rr * sn - ri * c;
        } else {        /* R e^{-i theta} */
            ar = rr * c + ri * sn;
            ai = ri * c - rr * sn;
        }
        const double scale = w[k] * cinc;
        const double s = st.s, t = st.t;
        const double wgt[4] = {(1.0 - t) * (1.0 - s), (1.0 - t) * s, t * (1.0 - s), t * s};
        for (int n = 0; n < 4; ++n) {
            const int64_t i = st.i0 + n / 2, q = st.j0 + n % 2;
            int64_t p = (i - N / 2) % N;
            if (p < 0) p += N;
            Are[p * NQ + q] += scale * wgt[n] * ar;
            Aim[p * NQ + q] += scale * wgt[n] * ai;
        }
    }
    /* sum over p for every (r, q): H[r][q] = sum_p A[p][q] W^{p (r - N/2)} */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        for (int64_t q = 0; q < NQ; ++q) {
            double sre = 0.0, sim = 0.0;
            for (int64_t p = 0; p < N; ++p) {
                int64_t kk = (p * (r - N / 2)) % N;
                if (kk < 0) kk += N;
                const double a = Are[p * NQ + q], b = Aim[p * NQ + q];
                sre += a * wr[kk] - b * wi[kk];
                sim += a * wi[kk] + b * wr[kk];
            }
            Hre[r * NQ + q] = sre;
            Him[r * NQ + q] = sim;
        }
    }
    /* g[r][c] = -2 Re sum_q H[r][q] W^{q (c - N/2)} */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        for (int64_t c = 0; c < N; ++c) {
            double sre = 0.0;
            for (int64_t q = 0; q < NQ; ++q) {
                int64_t kk = (q * (c - N / 2)) % N;
                if (kk < 0) kk += N;
                sre += Hre[r * NQ + q] * wr[kk] - Him[r * NQ + q] * wi[kk];
            }
            grad[r * N + c] = -2.0 * sre;
        }
    }
    free(Are); free(Aim); free(Hre); free(Him); free(wr); free(wi);
    return bad;
}

/* Gradient with respect to the profile values I_j, by the chain rule through
 * orc_sweep: every pixel passes its image gradient to the two radial samples
 * it interpolates, weighted dxy^2 (1 - f) and dxy^2 f; the centre pixel
 * passes dxy^2 (1 + Rmin/dR) to I_0 and -dxy^2 Rmin/dR to I_1. */
int orc_grad_profile(const double *gimg, int64_t Nr, double Rmin, double dR,
                     int64_t N, double dxy, double inc, double *gI)
{
    if (Nr < 2 || N < 2 || (N % 2) != 0) return -2;
    const double cos_inc = cos(inc);
    const double pix_area = dxy * dxy;
    const double t_max = (double)(Nr - 1);
    for (int64_t j = 0; j < Nr; ++j) gI[j] = 0.0;
    for (int64_t r = 0; r < N; ++r) {
        const double y = (double)(N / 2 - r) * dxy;
        for (int64_t c = 0; c < N; ++c) {
            if (r == N / 2 && c == N / 2) continue;
            const double x = (double)(N / 2 - c) * dxy;
            const double xs = x / cos_inc;
            const double rho = sqrt(xs * xs + y * y);
            const double t = (rho - Rmin) / dR;
            if (t >= 0.0 && t <= t_max) {
                int64_t j = (int64_t)floor(t);
                if (j > Nr - 2) j = Nr - 2;
                const double f = t - (double)j;
                gI[j] += gimg[r * N + c] * pix_area * (1.0 - f);
                gI[j + 1] += gimg[r * N + c] * pix_area * f;
            }
        }
    }
    const double gc = gimg[(N / 2) * N + (N / 2)];
    gI[0] += gc * pix_area * (1.0 + Rmin / dR);
    gI[1] += gc * pix_area * (-Rmin / dR);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Derivative of the swept image with respect to the inclination (the tilt
 * of orc_sweep): with rho = sqrt((x / cos inc)^2 + y^2) and the profile
 * linear on [r_j, r_{j+1}], d img / d inc = dxy^2 (I_{j+1} - I_j) / dR *
 * d rho / d inc, d rho / d inc = (x / cos inc)^2 tan(inc) / rho, on the same
 * segment j that orc_sweep uses; 0 outside the profile's range and at the
 * centre pixel (whose extrapolated value does not depend on inc).  Not in the
 * paper: the inclination gradient of a swept profile is the transform of
 * this image. */
int orc_sweep_dinc(const double *I, int64_t Nr, double Rmin, double dR, int64_t N,
                   double dxy, double inc, double *dimg)
{
    if (Nr < 2 || N < 2 || (N % 2) != 0) return -2;
    if (!(dR > 0.0) || !(dxy > 0.0) || !(cos(inc) > 0.0) || !(Rmin >= 0.0)) return -4;
    const double cos_inc = cos(inc), tan_inc = tan(inc);
    const double pix_area = dxy * dxy;
    const double t_max = (double)(Nr - 1);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        const double y = (double)(N / 2 - r) * dxy;
        for (int64_t c = 0; c < N; ++c) {
            const double x = (double)(N / 2 - c) * dxy;
            const double xs = x / cos_inc;
            const double rho = sqrt(xs * xs + y * y);
            const double t = (rho - Rmin) / dR;
            double val = 0.0;
            if (rho > 0.0 && t >= 0.0 && t <= t_max) {
                int64_t j = (int64_t)floor(t);
                if (j > Nr - 2) j = Nr - 2;
                val = (I[j + 1] - I[j]) / dR * (xs * xs * tan_inc / rho);
            }
            dimg[r * N + c] = val * pix_area;
        }
    }
    dimg[(N / 2) * N + (N / 2)] = 0.0;
    return 0;
}

/* chi^2 and its derivatives with respect to the geometry (not in the paper):
 * out5 = {chi2, d/dPA, d/d dRA, d/d dDec, d/d inc}.  With R = Vobs - V,
 * d chi2 / d a = -2 sum_k w_k Re(conj(R_k) dV_k / d a), and, following the
 * steps of orc_locate / orc_finish:
 *   - dV/d dRA = 2 pi i u V, dV/d dDec = 2 pi i v V (the phase);
 *   - PA moves the sampling point: u' = u cos PA - v sin PA and
 *     v' = u sin PA + v cos PA give du'/dPA = -v', dv'/dPA = u'; the point's
 *     grid coordinates are fu = m u' cinc / du and fv = m v' / du (m = -1 for
 *     mirrored points), and the bilinear value B(s, t) has
 *     dB/ds = (1-t)(b01 - b00) + t(b11 - b10), dB/dt = (1-s)(b10 - b00) + s(b11 - b01);
 *   - inc (image form, A-15): V^ = cinc conj_m(B(fu, fv)) with
 *     dfu/dinc = -m u' sin(inc) / du;
 *   - inc (swept profile, Gt != NULL, sampled with cinc = 1): the image
 *     itself depends on inc, and dV/dinc samples the spectrum Gt of
 *     orc_sweep_dinc's image at the same stencil.
 * Invalid points make chi2 NaN.  Sums in long double, in index order. */
int64_t orc_geograd(const double *G, const double *Gt, int64_t N, double dxy, const double *u,
                    const double *v, const double *re, const double *im, const double *w,
                    int64_t M, double PA, double dRA, double dDec, double inc, double *out5)
{
    const double du = 1.0 / ((double)N * dxy);
    const double cpa = cos(PA), spa = sin(PA);
    const double cinc = Gt ? 1.0 : cos(inc), sinc = Gt ? 0.0 : sin(inc);
    long double acc[5] = {0.0L, 0.0L, 0.0L, 0.0L, 0.0L};
    int64_t bad = 0;
    for (int64_t k = 0; k < M; ++k) {
        orc_stencil st;
        if (!orc_locate(u[k], v[k], N, du, cpa, spa, cinc, &st)) {
            bad += 1;
            continue;
        }
        double b[8];
        orc_shifted(G, N, st.i0, st.j0, &b[0], &b[1]);
        orc_shifted(G, N, st.i0, st.j0 + 1, &b[2], &b[3]);
        orc_shifted(G, N, st.i0 + 1, st.j0, &b[4], &b[5]);
        orc_shifted(G, N, st.i0 + 1, st.j0 + 1, &b[6], &b[7]);
        const double s = st.s, t = st.t;
        const double msign = st.conj ? -1.0 : 1.0;
        /* B and its partial derivatives (complex), before the mirror's conjugation */
        double Br = (1 - t) * ((1 - s) * b[0] + s * b[2]) + t * ((1 - s) * b[4] + s * b[6]);
        double Bi = (1 - t) * ((1 - s) * b[1] + s * b[3]) + t * ((1 - s) * b[5] + s * b[7]);
        double Bsr = (1 - t) * (b[2] - b[0]) + t * (b[6] - b[4]);
        double Bsi = (1 - t) * (b[3] - b[1]) + t * (b[7] - b[5]);
        double Btr = (1 - s) * (b[4] - b[0]) + s * (b[6] - b[2]);
        double Bti = (1 - s) * (b[5] - b[1]) + s * (b[7] - b[3]);
        if (st.conj) {
            Bi = -Bi;
            Bsi = -Bsi;
            Bti = -Bti;
        }
        const double up = u[k] * cpa - v[k] * spa, vp = u[k] * spa + v[k] * cpa;
        const double dfu_dpa = msign * cinc * (-vp) / du, dfv_dpa = msign * up / du;
        /* V^ and its derivatives (before the phase) */
        const double Vr = cinc * Br, Vi = cinc * Bi;
        const double Pr = cinc * (Bsr * dfu_dpa + Btr * dfv_dpa);
        const double Pi = cinc * (Bsi * dfu_dpa + Bti * dfv_dpa);
        double Ir, Ii;
        if (Gt) {
            double c[8];
            orc_shifted(Gt, N, st.i0, st.j0, &c[0], &c[1]);
            orc_shifted(Gt, N, st.i0, st.j0 + 1, &c[2], &c[3]);
            orc_shifted(Gt, N, st.i0 + 1, st.j0, &c[4], &c[5]);
            orc_shifted(Gt, N, st.i0 + 1, st.j0 + 1, &c[6], &c[7]);
            Ir = (1 - t) * ((1 - s) * c[0] + s * c[2]) + t * ((1 - s) * c[4] + s * c[6]);
            Ii = (1 - t) * ((1 - s) * c[1] + s * c[3]) + t * ((1 - s) * c[5] + s * c[7]);
            if (st.conj) Ii = -Ii;
        } else {
            const double dfu_dinc = -msign * up * sinc / du;
            Ir = -sinc * Br + cinc * Bsr * dfu_dinc;
            Ii = -sinc * Bi + cinc * Bsi * dfu_dinc;
        }
        /* the phase exp(i theta) */
        const double theta = TWO_PI * (u[k] * dRA + v[k] * dDec);
        const double cs = cos(theta), sn = sin(theta);
        const double VVr = Vr * cs - Vi * sn, VVi = Vr * sn + Vi * cs;
        const double Rr = re[k] - VVr, Ri = im[k] - VVi;
        /* Re(conj(R) z e^{i theta}) for each derivative z of V^ */
        const double Pr2 = Pr * cs - Pi * sn, Pi2 = Pr * sn + Pi * cs;
        const double Ir2 = Ir * cs - Ii * sn, Ii2 = Ir * sn + Ii * cs;
        /* dV/d dRA = i 2 pi u V: Re(conj(R) i X) = -Im(conj(R) X) = -(Rr Xi - Ri Xr) */
        const double imRV = Rr * VVi - Ri * VVr;
        acc[0] += (long double)(w[k] * (Rr * Rr + Ri * Ri));
        acc[1] += (long double)(-2.0 * w[k] * (Rr * Pr2 + Ri * Pi2));
        acc[2] += (long double)(-2.0 * w[k] * (-TWO_PI * u[k] * imRV));
        acc[3] += (long double)(-2.0 * w[k] * (-TWO_PI * v[k] * imRV));
        acc[4] += (long double)(-2.0 * w[k] * (Rr * Ir2 + Ri * Ii2));
    }
    for (int k = 0; k < 5; ++k) out5[k] = (double)acc[k];
    if (bad) out5[0] = NAN;
    return bad;
}
