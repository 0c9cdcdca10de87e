// kernels.h -- the gfx950 kernels of the visibility / chi-square path.
//
//   k_rows    image row (or swept profile row) -> real-to-complex FFT along x,
//             origin shift folded in as the output sign (-1)^q, written
//             transposed (column q contiguous) for the second pass.
//   k_cols    complex FFT along y of every needed column q, origin shift as
//             the sign (-1)^p, written back in place as the rows
//             p~ in [-P, P] that the uv points can reach.
//   k_sample  uv rotation, mirror, bilinear gather, deprojection, phase
//             shift; writes V or per-block partial sums of the weighted
//             chi^2, which k_reduce adds in a fixed order.
//
// Shifting the image origin to pixel (N/2, N/2) multiplies the unshifted
// DFT F[p][q] by exp(i pi (p + q)) = (-1)^(p+q) (Sec. 4 shift -> FFT -> shift),
// so no data is moved for it.
#pragma once
#include "fft_block.h"
#include "wave.h"

namespace gal {

extern __device__ c2<double> g_tw_d[2 * TW_MAX];
extern __device__ c2<float> g_tw_f[2 * TW_MAX];

template <typename T>
__device__ __forceinline__ const c2<T> *twiddles();
template <>
__device__ __forceinline__ const c2<double> *twiddles<double>() { return g_tw_d; }
template <>
__device__ __forceinline__ const c2<float> *twiddles<float>() { return g_tw_f; }

// Pointers read from device tables are generic, and loads through them
// become flat instructions; arrays known to be in device global memory are
// re-typed so that they load with global instructions.
template <typename T>
using gptr = const T __attribute__((address_space(1))) *;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const void *p) {
    return (gptr<T>)p;
}

// sin(pi x) and cos(pi x) of x = y / 128 for the phase factor of a uv point,
// by table and series: n = rint(y) and r = (y - n) / 128, |r| <= 1/256 (y - n
// is exact); (cos, -sin)(pi n / 128) is entry n mod 256 of the length-256
// twiddle row (exp(-2 pi i m / 256), stored at [256, 512)); sin and cos of
// z = pi r by their Taylor series through z^5 and z^6 (|z| <= pi/256:
// truncation below 1e-17); then the angle-addition formulas.  About 15 FP64
// operations and one cached 16-byte load; abs. error a few 1e-16.  The table
// index is exact for |y| < 2^51, i.e. phases |u dRA + v dDec| below 2^43
// turns; a NaN y reads some entry in range and gives a NaN phase.
__device__ __forceinline__ void sincospi_tab(double y, double &sn, double &cs) {
    const double n = rint(y);
    // n mod 256: n + 1.5 2^52 holds n in the low bits of its significand
    // (two's complement), whatever the sign of n
    const uint32_t idx = (uint32_t)__double_as_longlong(n + 6755399441055744.0) & 255u;
    const c2<double> t = *(const c2<double> *)((const char *)(g_tw_d + 256) + idx * 16u);
    const double z = (y - n) * (3.141592653589793 / 128.0);
    const double z2 = z * z;
    const double sb = fma(z * z2, fma(z2, 1.0 / 120.0, -1.0 / 6.0), z);
    const double cb = fma(z2, fma(z2, fma(z2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    sn = fma(-t.y, cb, t.x * sb);
    cs = fma(t.x, cb, t.y * sb);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous range of logical blocks so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    constexpr int NX = 8;
    const int q = nblk / NX, r = nblk % NX;
    const int x = bid % NX, l = bid / NX;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// ---------------------------------------------------------------------------
// geometry of one transform
struct Geom {
    int N;    // image side
    int Q;    // columns q in [0, Q) are transformed
    int P;    // rows p~ in [-P, P] are kept: stored row i = p~ + P
    int CS;   // stride (complex elements) between stored columns
};

// sweep of a radial profile (Sec. 2.2, Sec. 4, App. D)
struct SweepArgs {
    int Nr;
    double Rmin, inv_dR, dxy, inv_cos, pix_area, tmax;
    double tan_inc;  // used by the inclination derivative of the sweep only
    double dxs, t0;  // dxy / cos(inc); -Rmin / dR
};

// Profile coordinate of a pixel radius, t = (rho - Rmin) / dR, in one
// rounding step (the forward sweep and its transpose use the same t).
__device__ __forceinline__ double sweep_t(double rho, const SweepArgs &a) {
    return fma(rho, a.inv_dR, a.t0);
}

// Square root of a squared pixel radius: x is a normal number well above
// 2^-767 (pixel sizes are >= 1e-100 rad, checked on the host), so the
// hardware reciprocal square root y = (1 + e) / sqrt(x) (|e| about 5e-8)
// needs none of the general routine's range scaling.  One Newton correction
// of g = x y, g + (x - g^2) y / 2 = sqrt(x) (1 - 3 e^2 / 2 + O(e^3)), leaves a
// relative error of a few 1e-15 in rho: the profile coordinate
// t = (rho - Rmin) / dR moves by a few 1e-15 of rho / dR (below 1e-10 of a
// bin for rho < 1e4 dR), and the sweep, continuous in t inside the profile's
// range, by that fraction of a bin's step.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y;
    const double d = fma(-g, g, x);
    return fma(d, 0.5 * y, g);
}

// PI: pointer to the profile (generic, or global for pointers read from tables)
// Branch-free, so that the profile loads of neighbouring pixels can be in
// flight together: the bin index is clamped in floating point (every load is
// in bounds, NaN included) and a pixel outside [Rmin, Rmin + (Nr-1) dR] is
// selected to 0.  The centre pixel's rule -- the first segment extrapolated
// to rho = 0 -- is the same interpolation at bin 0 with t = -Rmin / dR <= 0:
// rho^2 is kept >= 1e-300 (every other pixel has rho^2 >= dxy^2 >= 1e-200), so
// there the root is 1e-150 instead of 0 and t differs by 1e-150 / dR.
template <typename PI>
__device__ __forceinline__ double sweep_pixel(PI I, int N, int r, int c, const SweepArgs &a) {
    const bool centre = (r == N / 2) && (c == N / 2);
    const double xs = (double)(N / 2 - c) * a.dxs;  // x / cos(inc)
    const double y = (double)(N / 2 - r) * a.dxy;
    const double rho = sqrt_pos(fmax(fma(xs, xs, y * y), 1e-300));
    const double t = sweep_t(rho, a);
    const uint32_t j = (uint32_t)(int)fmin(fmax(t, 0.0), (double)(a.Nr - 2));
    const double f = t - (double)j;
    // a multiply by 0 or 1 rather than a select, which the compiler would
    // turn back into a branch around the loads' use
    const double m = (centre || (t >= 0.0 && t <= a.tmax)) ? a.pix_area : 0.0;
    const auto Ij = I + j;  // I[j], I[j + 1]: one 16-byte load
    const double I0 = (double)Ij[0], I1 = (double)Ij[1];
    return fma(f, I1 - I0, I0) * m;
}

// A pixel other than the centre one, from its stretched abscissa xs = x /
// cos(inc) and the square of its ordinate: rho^2 >= dxy^2 there.  The same
// value as sweep_pixel with one clamp: tc is t clamped to the profile's
// range, the pixel is inside exactly when tc == t (NaN included: it is not).
template <typename PI>
__device__ __forceinline__ double sweep_px(PI I, double xs, double y2, const SweepArgs &a) {
    const double rho = sqrt_pos(fma(xs, xs, y2));
    const double t = sweep_t(rho, a);
    const double tc = fmin(fmax(t, 0.0), a.tmax);
    const uint32_t j = min((uint32_t)(int)tc, (uint32_t)(a.Nr - 2));
    const double f = tc - (double)j;
    const double m = (tc == t) ? a.pix_area : 0.0;
    const auto Ij = I + j;  // I[j], I[j + 1]: one 16-byte load
    const double I0 = (double)Ij[0], I1 = (double)Ij[1];
    return fma(f, I1 - I0, I0) * m;
}

// d pixel / d inc of the sweep (not in the paper): on the segment that
// sweep_pixel interpolates, (I[j+1] - I[j]) / dR times d rho / d inc =
// (x / cos inc)^2 tan(inc) / rho, times dxy^2; 0 outside the profile and at
// the centre pixel (its extrapolated value does not depend on inc).
template <typename PI>
__device__ __forceinline__ double sweep_pixel_dinc(PI I, int N, int r, int c, const SweepArgs &a) {
    const bool centre = (r == N / 2) && (c == N / 2);
    const double xs = (double)(N / 2 - c) * a.dxs;  // as sweep_pixel
    const double y = (double)(N / 2 - r) * a.dxy;
    const double rho = sqrt_pos(fmax(fma(xs, xs, y * y), 1e-300));
    const double t = sweep_t(rho, a);
    const uint32_t j = (uint32_t)(int)fmin(fmax(t, 0.0), (double)(a.Nr - 2));
    const double v = ((double)I[j + 1] - (double)I[j]) * a.inv_dR *
                     (xs * xs * a.tan_inc / rho) * a.pix_area;
    return (!centre && t >= 0.0 && t <= a.tmax) ? v : 0.0;
}

// ---------------------------------------------------------------------------
// Row pass.  Block of B rows, each a length-N real FFT done as a length-N/2
// complex FFT of z[n] = x[2n] + i x[2n+1] followed by the split
//   X[q] = (Z[q] + conj Z[L-q]) / 2 - i W_N^q (Z[q] - conj Z[L-q]) / 2.
// Output XT[q * CS + r] = (-1)^q X_r[q] for q < Q.
template <typename T, typename Cfg, bool PROFILE>
__device__ __forceinline__ void rows_body(const T *__restrict__ src, const SweepArgs &sw,
                                          const Geom &g, c2<T> *__restrict__ XT, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = 2 * L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int r0 = blk * B;

    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
        const int r = r0 + b;
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            if constexpr (PROFILE) {
                v[i * R0 + t].x = (T)sweep_pixel(src, N, r, 2 * n, sw);
                v[i * R0 + t].y = (T)sweep_pixel(src, N, r, 2 * n + 1, sw);
            } else {
                v[i * R0 + t] = *reinterpret_cast<const c2<T> *>(src + (size_t)r * N + 2 * n);
            }
        }
    }
    const c2<T> *tw = twiddles<T>();
    fft_passes<Cfg, 1>(v, lds, tw, tid);

    const c2<T> *wN = tw + N;  // exp(-2 pi i q / N)
    const T half = T(0.5);
    for (int idx = tid; idx < g.Q * B; idx += NT) {
        const int q = idx / B, b = idx % B;
        const c2<T> zk = lds[Cfg::at(b, q & (L - 1))];
        const c2<T> zc = cconj(lds[Cfg::at(b, (L - q) & (L - 1))]);
        const c2<T> s = cadd(zk, zc);
        const c2<T> d = cmul(wN[q], csub(zk, zc));
        c2<T> X = {half * (s.x + d.y), half * (s.y - d.x)};
        if (q & 1) X = {-X.x, -X.y};
        XT[(size_t)q * g.CS + r0 + b] = X;
    }
}

template <typename T, typename Cfg, bool PROFILE>
__global__ __launch_bounds__(Cfg::NT) void k_rows(const T *__restrict__ src, SweepArgs sw,
                                                  Geom g, c2<T> *__restrict__ XT) {
    rows_body<T, Cfg, PROFILE>(src, sw, g, XT, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Column pass, in place.  Block of B columns q0..q0+B-1, each a length-N
// complex FFT over the rows; output rows i in [0, 2P] hold p~ = i - P with
// sign (-1)^p~.
template <typename T, typename Cfg>
__device__ __forceinline__ void cols_body(const Geom &g, c2<T> *__restrict__ XT, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int q0 = blk * B;
    if (q0 >= g.Q) return;

    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
        const int q = q0 + b;
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            v[i * R0 + t] = (q < g.Q) ? XT[(size_t)q * g.CS + n] : c2<T>{T(0), T(0)};
        }
    }
    fft_passes<Cfg, 1>(v, lds, twiddles<T>(), tid);

    const int NPo = 2 * g.P + 1;
    for (int idx = tid; idx < NPo * B; idx += NT) {
        const int b = idx / NPo, i = idx % NPo;
        const int q = q0 + b;
        if (q >= g.Q) continue;
        const int pt = i - g.P;
        const int p = pt < 0 ? pt + L : pt;
        c2<T> X = lds[Cfg::at(b, p)];
        if (pt & 1) X = {-X.x, -X.y};
        XT[(size_t)q * g.CS + i] = X;
    }
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_cols(Geom g, c2<T> *__restrict__ XT) {
    cols_body<T, Cfg>(g, XT, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Swept profiles.  The swept image is even about its centre pixel in both
// axes: x_c = (N/2 - c) dxy and x_{N-c} = -x_c exactly, and rho depends on
// x^2 and y^2 only, so f[r][c] = f[r][N-c] and f[r][c] = f[N-r][c] bit for
// bit.  In DFT terms (indices mod N about the centre) the image is even, its
// shifted half spectrum G is real and even in p, and rows r and N - r have
// the same transform.  The two passes below use that: rows r in [0, N/2]
// only, two at a time as the real and imaginary parts of one length-N
// complex FFT (both transforms are real, so Re and Im separate them), a real
// intermediate, columns two at a time the same way, and a real spectrum
// stored for p in [0, P].  The samples equal those of the general path up
// to rounding.
//
// Row pass: pair m holds rows 2m and 2m+1; output XR[q * CS + r] (real,
// shift sign (-1)^q) for r in [0, N/2], q in [0, Qe) (Qe = Q rounded up to
// even so that the column pass can pair columns).
// TANGENT: the image swept is d image / d inc (sweep_pixel_dinc)
template <typename T, typename Cfg, typename PI = const T *__restrict__, bool TANGENT = false>
__device__ __forceinline__ void rows_sym_body(PI I, const SweepArgs &sw, const Geom &g, int Qe,
                                              T *__restrict__ XR, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int m0 = blk * B;

    // columns c and N - c hold the same pixel: sweep c in [0, N/2) into LDS
    // (no centre pixel there), then column N/2 with the centre pixel's rule
    constexpr int NH = N / 2;
    for (int idx = tid; idx < B * NH; idx += NT) {
        const int b = idx / NH, c = idx % NH;
        const int r = 2 * (m0 + b);  // rows r, r + 1 (r + 1 < N)
        if constexpr (TANGENT) {
            lds[Cfg::at(b, c)] = c2<T>{(T)sweep_pixel_dinc(I, N, r, c, sw),
                                       (T)sweep_pixel_dinc(I, N, r + 1, c, sw)};
        } else {
            const double xs = (double)(N / 2 - c) * sw.dxs;
            const double y0 = (double)(N / 2 - r) * sw.dxy, y1 = (double)(N / 2 - r - 1) * sw.dxy;
            lds[Cfg::at(b, c)] = c2<T>{(T)sweep_px(I, xs, y0 * y0, sw), (T)sweep_px(I, xs, y1 * y1, sw)};
        }
    }
    if (tid < B) {
        const int r = 2 * (m0 + tid);
        if constexpr (TANGENT)
            lds[Cfg::at(tid, NH)] = c2<T>{(T)sweep_pixel_dinc(I, N, r, NH, sw),
                                          (T)sweep_pixel_dinc(I, N, r + 1, NH, sw)};
        else
            lds[Cfg::at(tid, NH)] = c2<T>{(T)sweep_pixel(I, N, r, NH, sw),
                                          (T)sweep_pixel(I, N, r + 1, NH, sw)};
    }
    __syncthreads();
    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            v[i * R0 + t] = lds[Cfg::at(b, n <= N / 2 ? n : N - n)];
        }
    }
    const c2<T> *tw = twiddles<T>();
    fft_passes_but_last<Cfg, 1>(v, lds, tw, tid);
    // last pass in registers: only outputs q < Qe are kept, and the two rows
    // of a pair are adjacent in XR (one 16-byte store; CS and r are even)
    fft_last_pass<Cfg>(v, tw, tid, Qe, [&](int b, int q, c2<T> z) {
        const int r = 2 * (m0 + b);
        if (r > N / 2) return;
        if (q & 1) z = c2<T>{-z.x, -z.y};
        if (r + 1 <= N / 2)
            *reinterpret_cast<c2<T> *>(XR + (size_t)q * g.CS + r) = z;
        else
            XR[(size_t)q * g.CS + r] = z.x;
    });
}

// Half-length transform of even sequences.  A real sequence x of length
// N = 2h that is even about 0, x[n] = x[N - n], has a real and even DFT, and
// X[k] for k <= h follows from one real DFT of length h (two sequences share
// one complex transform as its real and imaginary parts).  With
//   a[n] = x[n] + x[h - n],  b[n] = x[n] - x[h - n]   (n in [0, h)),
// the even outputs are the (real) DFT of a, X[2m] = sum_n a[n] cos(2 pi n m / h),
// and the odd ones X[2m+1] = sum_n b[n] cos(pi n (2m+1) / h) obey
//   X[2m+1] - X[2m-1] = -2 sum_n b[n] sin(pi n / h) sin(2 pi n m / h),
// the (imaginary) DFT of the odd sequence b[n] sin(pi n / h).  So with
//   y[n] = a[n] + sin(pi n / h) b[n],  Y = DFT_h(y):
//   X[2m] = Re Y[m],  X[2m+1] = X[1] + 2 sum_{j=1..m} Im Y[j],
//   X[1] = sum_n b[n] cos(pi n / h).
// Half the FFT work of the length-N transform; the odd outputs come from a
// prefix sum (in FP64) over the kept outputs.
//
// The block's B pairs hold x[n], n in [0, h), at lds[Cfg::at(b, n)] and x[h]
// at xh[b] (one sequence in .x, the other in .y), staged by the caller and
// followed by a barrier.  For every pair b with active(b) and m in [0, Mk),
// out(b, m, ev, od) receives ev = X[2m] and od = -X[2m+1] of both sequences.
// The outputs of a pair are taken by one wave, or with SPREAD (B = 1 only)
// by every thread of the block: contiguous runs of m per thread, the odd
// outputs' prefix sum then crossing the waves through LDS (one more barrier;
// active(0) must then hold for the whole block or for none of it).
template <typename T, typename Cfg, bool SPREAD = false, typename Active, typename Out>
__device__ __forceinline__ void even_transform(c2<T> *lds, const c2<T> *xh, c2<double> *part,
                                               int tid, int Mk, Active active, Out out) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int H = L, N = 2 * L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    constexpr int NW = NT >= 64 ? NT / 64 : 1;
    const c2<T> *tw = twiddles<T>();
    const c2<T> *wN = tw + N;  // exp(-2 pi i n / N) = (cos(pi n / h), -sin(pi n / h))
    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;  // butterfly gi = b * LR + j of the first pass
        const int b = gi / LR, j = gi % LR;
        double p1 = 0.0, p2 = 0.0;
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            const c2<T> xa = lds[Cfg::at(b, n)];
            const c2<T> xb = n == 0 ? xh[b] : lds[Cfg::at(b, H - n)];
            const c2<T> w = wN[n];
            const T b1 = xa.x - xb.x, b2 = xa.y - xb.y;
            v[i * R0 + t] = c2<T>{xa.x + xb.x - w.y * b1, xa.y + xb.y - w.y * b2};
            p1 += (double)w.x * (double)b1;
            p2 += (double)w.x * (double)b2;
        }
        part[gi] = c2<double>{p1, p2};
    }
    // (the first pass's barrier orders these LDS reads before its writes)
    fft_passes<Cfg, 1>(v, lds, tw, tid);

    // one wave per pair: X[1] in a fixed order, then the outputs with the
    // prefix sum of the odd ones over contiguous runs of m per lane
    const int wave = tid >> 6, lane = tid & 63;
    if constexpr (SPREAD) {
        static_assert(B == 1, "SPREAD: one pair per block");
        __shared__ c2<double> wtot[NW];  // run sums of each wave
        if (!active(0)) return;
        double x1 = 0.0, x2 = 0.0;  // X[1], the same in every wave
        for (int k = lane; k < LR; k += 64) {
            x1 += part[k].x;
            x2 += part[k].y;
        }
        x1 = wave_sum(x1);
        x2 = wave_sum(x2);
        const int ch = (Mk + NT - 1) / NT;
        const int mb = min(tid * ch, Mk), me = min(mb + ch, Mk);
        double t1 = 0.0, t2 = 0.0;
        for (int m = mb; m < me; ++m) {
            const c2<T> z = lds[Cfg::at(0, m)], zc = lds[Cfg::at(0, (H - m) & (H - 1))];
            t1 += (double)z.y - (double)zc.y;
            t2 += (double)zc.x - (double)z.x;
        }
        const double e1 = wave_excl_scan(t1), e2 = wave_excl_scan(t2);
        if (lane == 63) wtot[wave] = c2<double>{e1 + t1, e2 + t2};
        __syncthreads();
        double b1 = 0.0, b2 = 0.0;
        for (int w = 0; w < wave; ++w) {
            b1 += wtot[w].x;
            b2 += wtot[w].y;
        }
        double a1 = x1 + (b1 + e1), a2 = x2 + (b2 + e2);
        for (int m = mb; m < me; ++m) {
            const c2<T> z = lds[Cfg::at(0, m)], zc = lds[Cfg::at(0, (H - m) & (H - 1))];
            a1 += (double)z.y - (double)zc.y;
            a2 += (double)zc.x - (double)z.x;
            const c2<T> ev{(T)(0.5 * ((double)z.x + (double)zc.x)),
                           (T)(0.5 * ((double)z.y + (double)zc.y))};
            const c2<T> od{(T)(-a1), (T)(-a2)};
            out(0, m, ev, od);
        }
        return;
    }
    const int ch = (Mk + 63) / 64;
    const int mb = lane * ch, me = min(mb + ch, Mk);
    for (int b = wave; b < B; b += NW) {
        if (!active(b)) continue;
        double x1 = 0.0, x2 = 0.0;
        for (int k = lane; k < LR; k += 64) {
            x1 += part[b * LR + k].x;
            x2 += part[b * LR + k].y;
        }
        x1 = wave_sum(x1);
        x2 = wave_sum(x2);
        // 2 Im Y[m] of each sequence from Z[m], Z[h - m] (Y1 = (Z[m] + conj Z[h-m]) / 2,
        // Y2 = (Z[m] - conj Z[h-m]) / 2i)
        double t1 = 0.0, t2 = 0.0;
        for (int m = mb; m < me; ++m) {
            const c2<T> z = lds[Cfg::at(b, m)], zc = lds[Cfg::at(b, (H - m) & (H - 1))];
            t1 += (double)z.y - (double)zc.y;
            t2 += (double)zc.x - (double)z.x;
        }
        double a1 = x1 + wave_excl_scan(t1), a2 = x2 + wave_excl_scan(t2);
        for (int m = mb; m < me; ++m) {
            const c2<T> z = lds[Cfg::at(b, m)], zc = lds[Cfg::at(b, (H - m) & (H - 1))];
            a1 += (double)z.y - (double)zc.y;
            a2 += (double)zc.x - (double)z.x;
            const c2<T> ev{(T)(0.5 * ((double)z.x + (double)zc.x)),
                           (T)(0.5 * ((double)z.y + (double)zc.y))};  // X[2m]
            const c2<T> od{(T)(-a1), (T)(-a2)};                       // -X[2m+1]
            out(b, m, ev, od);
        }
    }
}

// Row pass of a swept profile by half-length transforms: every row of the
// (centred) swept image is even, so even_transform applies to the row pairs.
// Half the FFT work of rows_sym_body, same output:
// XR[q * CS + r] = (-1)^q X_r[q], q < Qe.
template <typename T, typename Cfg, typename PI, bool TANGENT = false>
__device__ __forceinline__ void rows_even_body(PI I, const SweepArgs &sw, const Geom &g, int Qe,
                                               T *__restrict__ XR, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int H = L, N = 2 * L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    __shared__ c2<T> xh[B];               // x[h] of each row pair
    __shared__ c2<double> part[B * LR];   // per-butterfly parts of X[1]
    const int tid = threadIdx.x;
    const int m0 = blk * B;

    // sweep: columns c in [0, h) (c and N - c hold the same pixel; no centre
    // pixel there), E per thread, then column h with the centre pixel's rule
    static_assert(B * H == E * NT, "sweep: E pixel pairs per thread");
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int idx = tid + k * NT;
        const int b = idx / H, c = idx % H;
        const int r = 2 * (m0 + b);  // rows r, r + 1
        if constexpr (TANGENT) {
            lds[Cfg::at(b, c)] = c2<T>{(T)sweep_pixel_dinc(I, N, r, c, sw),
                                       (T)sweep_pixel_dinc(I, N, r + 1, c, sw)};
        } else {
            const double xs = (double)(N / 2 - c) * sw.dxs;
            const double y0 = (double)(N / 2 - r) * sw.dxy, y1 = (double)(N / 2 - r - 1) * sw.dxy;
            lds[Cfg::at(b, c)] = c2<T>{(T)sweep_px(I, xs, y0 * y0, sw), (T)sweep_px(I, xs, y1 * y1, sw)};
        }
    }
    if (tid < B) {
        const int r = 2 * (m0 + tid);
        if constexpr (TANGENT)
            xh[tid] = c2<T>{(T)sweep_pixel_dinc(I, N, r, H, sw), (T)sweep_pixel_dinc(I, N, r + 1, H, sw)};
        else
            xh[tid] = c2<T>{(T)sweep_pixel(I, N, r, H, sw), (T)sweep_pixel(I, N, r + 1, H, sw)};
    }
    __syncthreads();
    // Qe even, <= h + 2: m in [0, Qe / 2) gives columns 2m and 2m + 1 < Qe
    even_transform<T, Cfg>(
        lds, xh, part, tid, Qe / 2, [&](int b) { return 2 * (m0 + b) <= N / 2; },
        [&](int b, int m, c2<T> ev, c2<T> od) {
            const int r = 2 * (m0 + b);
            T *dst = XR + (size_t)(2 * m) * g.CS + r;
            if (r + 1 <= N / 2) {
                *reinterpret_cast<c2<T> *>(dst) = ev;
                *reinterpret_cast<c2<T> *>(dst + g.CS) = od;
            } else {
                dst[0] = ev.x;
                dst[g.CS] = od.x;
            }
        });
}

template <typename T, typename Cfg, bool TANGENT = false>
__global__ __launch_bounds__(Cfg::NT) void k_rows_even(const T *__restrict__ I, SweepArgs sw,
                                                       Geom g, int Qe, T *__restrict__ XR) {
    rows_even_body<T, Cfg, const T *__restrict__, TANGENT>(I, sw, g, Qe, XR,
                                                           xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, typename Cfg, bool TANGENT = false>
__global__ __launch_bounds__(Cfg::NT) void k_rows_sym(const T *__restrict__ I, SweepArgs sw,
                                                      Geom g, int Qe, T *__restrict__ XR) {
    rows_sym_body<T, Cfg, const T *__restrict__, TANGENT>(I, sw, g, Qe, XR,
                                                          xcd_remap(blockIdx.x, gridDim.x));
}

// Column pass of a swept profile, in place: pair of columns (2m, 2m+1),
// input over r in [0, N) from the stored half r' = min(r, N - r); output
// SR[q * CS + p] = (-1)^p G[p][q] for p in [0, P].
template <typename T, typename Cfg>
__device__ __forceinline__ void cols_sym_body(const Geom &g, int Qe, T *__restrict__ XR, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int m0 = blk * B;
    if (2 * m0 >= Qe) return;

    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
        const int q = 2 * (m0 + b);
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            const int rr = n <= N / 2 ? n : N - n;
            if (q < Qe) {
                v[i * R0 + t].x = XR[(size_t)q * g.CS + rr];
                v[i * R0 + t].y = XR[(size_t)(q + 1) * g.CS + rr];
            } else {
                v[i * R0 + t] = c2<T>{T(0), T(0)};
            }
        }
    }
    const c2<T> *tw = twiddles<T>();
    fft_passes_but_last<Cfg, 1>(v, lds, tw, tid);
    // last pass in registers, rows p <= P kept; every read of this block's
    // columns happened before the first barrier, so the in-place stores are safe
    fft_last_pass<Cfg>(v, tw, tid, g.P + 1, [&](int b, int p, c2<T> z) {
        const int q = 2 * (m0 + b);
        if (q >= Qe) return;
        const T sg = (p & 1) ? T(-1) : T(1);
        XR[(size_t)q * g.CS + p] = sg * z.x;
        XR[(size_t)(q + 1) * g.CS + p] = sg * z.y;
    });
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_cols_sym(Geom g, int Qe, T *__restrict__ XR) {
    cols_sym_body<T, Cfg>(g, Qe, XR, blockIdx.x);
}

// Column pass of a swept profile by half-length transforms, for images whose
// full-length column does not fit in LDS (16384^2 in FP64).  A column of the
// row pass's output is even in r about 0 (stored half r in [0, N/2]), so
// even_transform applies with x[n] read from XR.  Columns q = 2 (m0 + b) and
// q + 1 are the two sequences of a pair.  In place, as cols_sym_body:
// SR[q * CS + p] = (-1)^p G[p][q] for p in [0, P] (every read of the block's
// columns happens before its first barrier).
template <typename T, typename Cfg>
__device__ __forceinline__ void cols_even_body(const Geom &g, int Qe, T *__restrict__ XR, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int H = L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    __shared__ c2<T> xh[B];
    __shared__ c2<double> part[B * LR];
    const int tid = threadIdx.x;
    const int m0 = blk * B;
    if (2 * m0 >= Qe) return;
    static_assert(B * H == E * NT, "E values per thread");
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int idx = tid + k * NT;
        const int b = idx / H, n = idx % H;
        const int q = 2 * (m0 + b);
        lds[Cfg::at(b, n)] = q < Qe ? c2<T>{XR[(size_t)q * g.CS + n], XR[(size_t)(q + 1) * g.CS + n]}
                                    : c2<T>{T(0), T(0)};
    }
    if (tid < B) {
        const int q = 2 * (m0 + tid);
        xh[tid] = q < Qe ? c2<T>{XR[(size_t)q * g.CS + H], XR[(size_t)(q + 1) * g.CS + H]}
                         : c2<T>{T(0), T(0)};
    }
    __syncthreads();
    // m in [0, P / 2 + 1): rows 2m <= P and 2m + 1 (kept when <= P)
    even_transform<T, Cfg>(
        lds, xh, part, tid, g.P / 2 + 1, [&](int b) { return 2 * (m0 + b) < Qe; },
        [&](int b, int m, c2<T> ev, c2<T> od) {
            T *dst = XR + (size_t)(2 * (m0 + b)) * g.CS + 2 * m;
            dst[0] = ev.x;
            dst[g.CS] = ev.y;
            if (2 * m + 1 <= g.P) {
                dst[1] = od.x;
                dst[g.CS + 1] = od.y;
            }
        });
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_cols_even(Geom g, int Qe, T *__restrict__ XR) {
    cols_even_body<T, Cfg>(g, Qe, XR, blockIdx.x);
}

// Column pass of a general image whose column does not fit in LDS (16384^2
// in FP64), in two launches by the four-step factorisation of the DFT: with
// n = n1 + N1 n2 and p = k2 + N2 k1 (N = N1 N2),
//   X[k2 + N2 k1] = sum_n1 W_N1^(n1 k1) [ W_N^(n1 k2) sum_n2 x[n1 + N1 n2] W_N2^(n2 k2) ],
// W_M = exp(-2 pi i / M).  Step A, in place: for a group of B values n1, the
// length-N2 DFTs over n2, times W_N^(n1 k2), stored at n1 + N1 k2.  Step B:
// for a group of B values k2, the length-N1 DFTs over n1 (contiguous in
// memory), whose outputs p~ in [-P, P] go to the separate spectrum
// SP[q * CS2 + p~ + P] with the shift sign (-1)^p~ (cols_body's layout).
// blockIdx.y = column q.  Cfg: B sequences of length N1 = N2.
template <typename T, typename Cfg, int NTOT>
__global__ __launch_bounds__(Cfg::NT) void k_cols4a(Geom g, c2<T> *__restrict__ XT) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N1 = NTOT / L;
    static_assert(N1 == L, "square factorisation");
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int n10 = blockIdx.x * B;
    c2<T> *col = XT + (size_t)blockIdx.y * g.CS;
    // x[n1 + N1 n2], n1 fastest: runs of B contiguous values
    for (int idx = tid; idx < B * L; idx += NT) {
        const int b = idx % B, n2 = idx / B;
        lds[Cfg::at(b, n2)] = col[n10 + b + (size_t)N1 * n2];
    }
    __syncthreads();
    c2<T> v[E];
    fft_gather<Cfg, 1>(v, lds, tid);
    const c2<T> *tw = twiddles<T>();
    fft_passes<Cfg, 1>(v, lds, tw, tid);
    const c2<T> *wN = tw + NTOT;  // exp(-2 pi i m / N)
    for (int idx = tid; idx < B * L; idx += NT) {
        const int b = idx % B, k2 = idx / B;
        const int n1 = n10 + b;
        col[n1 + (size_t)N1 * k2] = cmul(lds[Cfg::at(b, k2)], wN[(n1 * k2) & (NTOT - 1)]);
    }
}

template <typename T, typename Cfg, int NTOT>
__global__ __launch_bounds__(Cfg::NT) void k_cols4b(Geom g, const c2<T> *__restrict__ XT,
                                                    c2<T> *__restrict__ SP, int CS2) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N2 = NTOT / L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int k20 = blockIdx.x * B;
    const c2<T> *col = XT + (size_t)blockIdx.y * g.CS;
    // first-pass inputs y[n1 + N1 k2] straight from memory (n1 contiguous)
    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
#pragma unroll
        for (int t = 0; t < R0; ++t) v[i * R0 + t] = col[j + t * LR + (size_t)L * (k20 + b)];
    }
    fft_passes<Cfg, 1>(v, lds, twiddles<T>(), tid);
    c2<T> *out = SP + (size_t)blockIdx.y * CS2;
    for (int idx = tid; idx < B * L; idx += NT) {
        const int b = idx % B, k1 = idx / B;
        const int p = k20 + b + N2 * k1;
        const int pt = p < NTOT / 2 ? p : p - NTOT;
        if (pt < -g.P || pt > g.P) continue;
        c2<T> X = lds[Cfg::at(b, k1)];
        if (pt & 1) X = c2<T>{-X.x, -X.y};
        out[pt + g.P] = X;
    }
}

// ---------------------------------------------------------------------------
// Sampling (Sec. 3.3, Sec. 3.4, App. D) and the chi^2 reduction (Sec. 3.1).
struct SampleArgs {
    int64_t M;
    double inv_du;             // N dxy
    double cpa, spa, cinc;     // cos PA, sin PA, cos inc
    double cpa_du, spa_du;     // cos PA, sin PA times N dxy (= 1 / du)
    double dRA, dDec;
    double ph_u, ph_v;         // 256 dRA, 256 dDec: 128 x 2 (u dRA + v dDec), exactly
    int jmax, imin, imax;      // valid stencil corners: j0 <= jmax, imin <= i0 <= imax
};

// exp(i theta) of a uv point, theta = 2 pi (u dRA + v dDec)
__device__ __forceinline__ void phase_of(const SampleArgs &a, double u, double v, double &sn,
                                         double &cs) {
    sincospi_tab(fma(u, a.ph_u, v * a.ph_v), sn, cs);
}

constexpr int SAMPLE_NT = 256;
constexpr int SAMPLE_PPT = 4;

struct Control {
    unsigned int reserved;
    int flag;              // status bits, set with atomicOr (see below)
};
// status bits of Control::flag
constexpr int STATUS_UV = 1;   // a uv point fell outside the spectrum (its V is NaN)
constexpr int STATUS_GEO = 2;  // a batch job's geometry row failed its checks (chi^2 NaN)

// Bilinear sample of the stored spectrum at one uv point: rotation by PA,
// deprojection, mirror of u' < 0 (conjugate), 4-node interpolation, flux
// factor cos(inc), phase exp(+2 pi i (u dRA + v dDec)).
template <typename T>
struct Stencil {
    const c2<T> *c0;   // node (q, i); (q, i+1) follows, (q+1, .) is CS further
    double s, t;
    bool mirror, ok;
    int q, i;          // c0 = S + q * CS + i
};

template <typename T>
__device__ __forceinline__ Stencil<T> locate(const c2<T> *__restrict__ S, const Geom &g,
                                             const SampleArgs &a, double u, double v) {
    Stencil<T> st;
    // grid coordinates of the rotated, deprojected point (1 / du folded into
    // the rotation)
    double fu = (u * a.cpa_du - v * a.spa_du) * a.cinc;
    double fv = u * a.spa_du + v * a.cpa_du;
    st.mirror = fu < 0.0;
    if (st.mirror) {
        fu = -fu;
        fv = -fv;
    }
    const double j0f = floor(fu), i0f = floor(fv);
    st.ok = (j0f >= 0.0) && (j0f <= (double)a.jmax) && (i0f >= (double)a.imin) &&
            (i0f <= (double)a.imax);
    st.s = fu - j0f;
    st.t = fv - i0f;
    const int q = st.ok ? (int)j0f : 0;
    const int i = st.ok ? (int)i0f + g.P : g.P;
    st.c0 = S + (size_t)q * g.CS + i;
    st.q = q;
    st.i = i;
    return st;
}

template <typename T>
__device__ __forceinline__ void finish(const Stencil<T> &st, c2<T> a00, c2<T> a10, c2<T> a01,
                                       c2<T> a11, const SampleArgs &a, double u, double v,
                                       double &Vre, double &Vim) {
    if (!st.ok) {
        Vre = __builtin_nan("");
        Vim = __builtin_nan("");
        return;
    }
    const double s = st.s, t = st.t;
    const double w00 = (1.0 - t) * (1.0 - s), w01 = (1.0 - t) * s;
    const double w10 = t * (1.0 - s), w11 = t * s;
    double br = w00 * (double)a00.x + w01 * (double)a01.x + w10 * (double)a10.x + w11 * (double)a11.x;
    double bi = w00 * (double)a00.y + w01 * (double)a01.y + w10 * (double)a10.y + w11 * (double)a11.y;
    if (st.mirror) bi = -bi;
    br *= a.cinc;
    bi *= a.cinc;
    // exp(i theta), theta = 2 pi (u dRA + v dDec)
    double sn, cs;
    phase_of(a, u, v, sn, cs);
    Vre = br * cs - bi * sn;
    Vim = br * sn + bi * cs;
}


// sum over the block in a fixed order; result valid in thread 0
__device__ __forceinline__ double block_sum(double x, double *red) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    }
    __syncthreads();
    return s;
}

// End of a chi^2 sampling block: the block's partial sum, added to the
// others in index order by k_reduce (bitwise repeatable).  A last-block
// reduction inside this kernel would need a device-scope release in every
// block, which on this chip writes back the L2 once per block and costs more
// than the second launch.
__device__ __forceinline__ void chi2_block_end(double acc, double *red, int blk,
                                               double *__restrict__ partials) {
    const double bs = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blk] = bs;
}

// Final chi^2: one block sums the per-block partials in a fixed order.
// Second stage of the chi^2 sum: one block of REDUCE_NT threads; thread t
// adds partials t, t + REDUCE_NT, ... in that order with all loads issued
// before the adds (a dependent chain of L2 round trips otherwise sets the
// kernel's time), then the block sum.  Bitwise repeatable.
constexpr int REDUCE_NT = 1024;
constexpr int REDUCE_UNROLL = 8;

__device__ __forceinline__ double strided_sum(const double *__restrict__ part, int n) {
    double s = 0.0;
    for (int k0 = threadIdx.x; k0 < n; k0 += REDUCE_NT * REDUCE_UNROLL) {
        double x[REDUCE_UNROLL];
#pragma unroll
        for (int u = 0; u < REDUCE_UNROLL; ++u) {
            const int k = k0 + u * REDUCE_NT;
            x[u] = k < n ? part[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < REDUCE_UNROLL; ++u) s += x[u];
    }
    return s;
}

__global__ __launch_bounds__(REDUCE_NT) void k_reduce(const double *__restrict__ partials, int n,
                                                      double *__restrict__ out) {
    __shared__ double red[REDUCE_NT / 64];
    const double tot = block_sum(strided_sum(partials, n), red);
    if (threadIdx.x == 0) *out = tot;
}

// Sampling of the real, p-even spectrum of a swept profile: node (q, p~)
// holds SR[q * CS + |p~|], so the two rows of a stencil are the adjacent
// pair starting at min(|p~0|, |p~0 + 1|).  Signed form, kept for the
// geometry gradient, whose derivatives follow the mirrored orientation.
template <typename T>
struct StencilR {
    const T *c0;       // SR + q * CS + lo; row lo and lo + 1
    double s, t;
    bool swap, ok;     // swap: node p~0 is at lo + 1 (p~0 < 0)
    int q, i;          // c0 = SR + q * CS + i (i = lo)
};

template <typename T>
__device__ __forceinline__ StencilR<T> locate_r(const T *__restrict__ S, const Geom &g,
                                                const SampleArgs &a, double u, double v) {
    StencilR<T> st;
    // real spectra are those of swept profiles, whose inclination is in the
    // swept image: they are sampled with cos(inc) = 1 (a.cinc is 1 here)
    double fu = u * a.cpa_du - v * a.spa_du;
    double fv = u * a.spa_du + v * a.cpa_du;
    if (fu < 0.0) {
        fu = -fu;
        fv = -fv;
    }
    const double j0f = floor(fu), i0f = floor(fv);
    st.ok = (j0f >= 0.0) && (j0f <= (double)a.jmax) && (i0f >= (double)a.imin) &&
            (i0f <= (double)a.imax);
    st.s = fu - j0f;
    st.t = fv - i0f;
    const int q = st.ok ? (int)j0f : 0;
    const int p0 = st.ok ? (int)i0f : 0;
    st.swap = p0 < 0;
    const int lo = st.swap ? -p0 - 1 : p0;
    st.c0 = S + (size_t)q * g.CS + lo;
    st.q = q;
    st.i = lo;
    return st;
}

// Even form, for the chi^2 samplers and the adjoint scatter.  The spectrum of
// a swept profile is real and even in u' and in v' separately (the disc
// before rotation is symmetric about both axes), and the piecewise-linear
// interpolant of an even node sequence is itself even: the bilinear value at
// (u', v') is the one at (|u'|, |v'|), read from the stored rows |p~| with
// neither mirror nor row swap.  Validity is the decision locate_r takes on
// the mirrored point (for integer bounds, floor(x) >= lo iff x >= lo and
// floor(x) <= hi iff x < hi + 1); an invalid point gets a clamped stencil
// inside the stored spectrum, whose value the caller discards.
template <typename T>
struct StencilE {
    uint32_t off;      // byte offset of node (q, i) from SR: (q * CS + i) sizeof(T), below
                       // 2^32 for N <= 8192; rows i and i + 1 are adjacent, column q + 1
                       // is CS elements further
    double s, t;       // weights of column q + 1 and of row i + 1
    bool ok;
    int q, i;
};

// The four node values of an even-form stencil: (q, i), (q, i+1), (q+1, i),
// (q+1, i+1).  A uniform base plus a 32-bit offset per lane.
template <typename T>
__device__ __forceinline__ void nodes_e(const T *__restrict__ S, const StencilE<T> &st, int CS,
                                        double &x0, double &x1, double &y0, double &y1) {
    const char *b = (const char *)S;
    const T *c = (const T *)(b + st.off);
    const T *d = (const T *)(b + (st.off + (uint32_t)CS * (uint32_t)sizeof(T)));
    x0 = c[0];
    x1 = c[1];
    y0 = d[0];
    y1 = d[1];
}

template <typename T>
__device__ __forceinline__ StencilE<T> locate_e(const Geom &g, const SampleArgs &a, double u,
                                                double v) {
    StencilE<T> st;
    const double fu = u * a.cpa_du - v * a.spa_du;
    const double fv = u * a.spa_du + v * a.cpa_du;
    const double fvm = fu < 0.0 ? -fv : fv;  // v' of the mirrored point
    const double au = fabs(fu), av = fabs(fv);
    st.ok = (au < (double)a.jmax + 1.0) && (fvm >= (double)a.imin) &&
            (fvm < (double)a.imax + 1.0);
    // lower nodes clamped to the last valid ones (NaN -> the clamp): rows up
    // to -imin = min(P, N/2) and columns up to jmax + 1 are stored
    const double qf = fmin(floor(au), (double)a.jmax);
    const double i0 = fmin(floor(av), (double)(-a.imin - 1));
    st.s = au - qf;
    st.t = av - i0;
    st.q = (int)qf;
    st.i = (int)i0;
    st.off = ((uint32_t)st.q * (uint32_t)g.CS + (uint32_t)st.i) * (uint32_t)sizeof(T);
    return st;
}

// Bilinear value from the four nodes (row i: a00, a01; row i + 1: a10, a11;
// second index the column).
__device__ __forceinline__ double bilerp(double a00, double a01, double a10, double a11, double s,
                                         double t) {
    const double b0 = fma(s, a01 - a00, a00), b1 = fma(s, a11 - a10, a10);
    return fma(t, b1 - b0, b0);
}

template <typename T, bool CHI2>
__global__ __launch_bounds__(SAMPLE_NT) void k_sample_sym(
    const T *__restrict__ S, Geom g, SampleArgs a, const T *__restrict__ u,
    const T *__restrict__ v, const T *__restrict__ re, const T *__restrict__ im,
    const T *__restrict__ w, c2<T> *__restrict__ vis, const int32_t *__restrict__ perm,
    double *__restrict__ partials, Control *ctl) {
    constexpr int PPT = SAMPLE_PPT;
    __shared__ double red[SAMPLE_NT / 64];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)blk * (SAMPLE_NT * PPT) + threadIdx.x;
    // every column load is issued before the arithmetic (the observations
    // are independent of the stencil, so they stream in during the gathers)
    double uu[PPT], vv[PPT], rr[PPT], ii[PPT], ww[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        const bool in = k < a.M;
        uu[p] = in ? (double)u[k] : 0.0;
        vv[p] = in ? (double)v[k] : 0.0;
        if constexpr (CHI2) {
            rr[p] = in ? (double)re[k] : 0.0;
            ii[p] = in ? (double)im[k] : 0.0;
            ww[p] = in ? (double)w[k] : 0.0;
        }
    }
    StencilE<T> st[PPT];
    double x0[PPT], x1[PPT], y0[PPT], y1[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        st[p] = locate_e<T>(g, a, uu[p], vv[p]);
        nodes_e<T>(S, st[p], g.CS, x0[p], x1[p], y0[p], y1[p]);
    }
    double acc = 0.0;
    bool bad = false;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        const bool in = k < a.M;
        double sn, cs;
        phase_of(a, uu[p], vv[p], sn, cs);
        double b = bilerp(x0[p], y0[p], x1[p], y1[p], st[p].s, st[p].t);
        b = st[p].ok ? b : __builtin_nan("");
        bad |= in && !st[p].ok;
        const double Vre = b * cs, Vim = b * sn;  // cos(inc) = 1 on real spectra
        if constexpr (CHI2) {
            // no branch on `in`: a point past M has w = 0 and a valid stencil
            const double dr = Vre - rr[p];
            const double di = Vim - ii[p];
            acc += ww[p] * (dr * dr + di * di);
        } else {
            if (in) vis[perm ? (int64_t)perm[k] : k] = c2<T>{(T)Vre, (T)Vim};
        }
    }
    if (bad) atomicOr(&ctl->flag, STATUS_UV);
    if constexpr (CHI2) chi2_block_end(acc, red, blk, partials);
}

// Each thread takes SAMPLE_PPT points strided by the block size: all loads
// are issued before the arithmetic.  CHI2: see chi2_block_end.
template <typename T, bool CHI2>
__global__ __launch_bounds__(SAMPLE_NT) void k_sample(
    const c2<T> *__restrict__ S, Geom g, SampleArgs a, const T *__restrict__ u,
    const T *__restrict__ v, const T *__restrict__ re, const T *__restrict__ im,
    const T *__restrict__ w, c2<T> *__restrict__ vis, const int32_t *__restrict__ perm,
    double *__restrict__ partials, Control *ctl) {
    constexpr int PPT = SAMPLE_PPT;
    __shared__ double red[SAMPLE_NT / 64];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)blk * (SAMPLE_NT * PPT) + threadIdx.x;
    // every column load is issued before the arithmetic (the observations
    // are independent of the stencil, so they stream in during the gathers)
    double uu[PPT], vv[PPT], rr[PPT], ii[PPT], ww[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        const bool in = k < a.M;
        uu[p] = in ? (double)u[k] : 0.0;
        vv[p] = in ? (double)v[k] : 0.0;
        if constexpr (CHI2) {
            rr[p] = in ? (double)re[k] : 0.0;
            ii[p] = in ? (double)im[k] : 0.0;
            ww[p] = in ? (double)w[k] : 0.0;
        }
    }
    Stencil<T> st[PPT];
    c2<T> n00[PPT], n10[PPT], n01[PPT], n11[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        st[p] = locate<T>(S, g, a, uu[p], vv[p]);
        n00[p] = st[p].c0[0];
        n10[p] = st[p].c0[1];
        n01[p] = st[p].c0[g.CS];
        n11[p] = st[p].c0[g.CS + 1];
    }
    double acc = 0.0;
    bool bad = false;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        if (k < a.M) {
            double Vre, Vim;
            finish<T>(st[p], n00[p], n10[p], n01[p], n11[p], a, uu[p], vv[p], Vre, Vim);
            bad |= !st[p].ok;
            if constexpr (CHI2) {
                const double dr = Vre - rr[p];
                const double di = Vim - ii[p];
                acc += ww[p] * (dr * dr + di * di);
            } else {
                vis[perm ? (int64_t)perm[k] : k] = c2<T>{(T)Vre, (T)Vim};
            }
        }
    }
    if (bad) atomicOr(&ctl->flag, STATUS_UV);
    if constexpr (CHI2) chi2_block_end(acc, red, blk, partials);
}


// ---------------------------------------------------------------------------
// stand-alone sweep (gal_sweep)
template <typename T>
__global__ __launch_bounds__(256) void k_sweep(const T *__restrict__ I, SweepArgs sw, int N,
                                               T *__restrict__ img) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int r = (int)(idx / N), c = (int)(idx % N);
    img[idx] = (T)sweep_pixel(I, N, r, c, sw);
}

// internal layout (column q, row i = p~ + P) <-> G[p][q] with P = N/2
template <typename T>
__global__ __launch_bounds__(256) void k_spec_out(const c2<T> *__restrict__ S, Geom g,
                                                  c2<T> *__restrict__ G) {
    const int NQ = g.N / 2 + 1;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)g.N * NQ) return;
    const int p = (int)(idx / NQ), q = (int)(idx % NQ);
    const int pt = p < g.N / 2 ? p : p - g.N;
    G[idx] = S[(size_t)q * g.CS + pt + g.P];
}

template <typename T>
__global__ __launch_bounds__(256) void k_spec_in(const c2<T> *__restrict__ G, Geom g,
                                                 c2<T> *__restrict__ S) {
    const int NQ = g.N / 2 + 1;
    const int NPo = 2 * g.P + 1;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)NQ * NPo) return;
    const int q = (int)(idx / NPo), i = (int)(idx % NPo);
    int p = (i - g.P) % g.N;
    if (p < 0) p += g.N;
    S[(size_t)q * g.CS + i] = G[(size_t)p * NQ + q];
}

__global__ void k_ctrl_zero(Control *ctl) {
    if (threadIdx.x == 0) {
        ctl->reserved = 0u;
        ctl->flag = 0;
    }
}

}  // namespace gal
