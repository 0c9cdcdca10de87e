// kernels.h -- the gfx950 kernels of the visibility / chi-square path.
//
//   k_rows    image row (or swept profile row) -> real-to-complex FFT along x,
//             origin shift folded in as the output sign (-1)^q, written
//             transposed (column q contiguous) for the second pass.
//   k_cols    complex FFT along y of every needed column q, origin shift as
//             the sign (-1)^p, written back in place as the rows
//             p~ in [-P, P] that the uv points can reach.
//   k_sample  uv rotation, mirror, bilinear gather, deprojection, phase
//             shift; writes V or reduces the weighted chi^2 (last-block
//             deterministic reduction).
//
// Shifting the image origin to pixel (N/2, N/2) multiplies the unshifted
// DFT F[p][q] by exp(i pi (p + q)) = (-1)^(p+q) (Sec. 4 shift -> FFT -> shift),
// so no data is moved for it.
#pragma once
#include "fft_block.h"

namespace gal {

extern __device__ c2<double> g_tw_d[2 * TW_MAX];
extern __device__ c2<float> g_tw_f[2 * TW_MAX];

template <typename T>
__device__ __forceinline__ const c2<T> *twiddles();
template <>
__device__ __forceinline__ const c2<double> *twiddles<double>() { return g_tw_d; }
template <>
__device__ __forceinline__ const c2<float> *twiddles<float>() { return g_tw_f; }

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
};

template <typename T>
__device__ __forceinline__ double sweep_pixel(const T *__restrict__ I, int N, int r, int c,
                                              const SweepArgs &a) {
    if (r == N / 2 && c == N / 2) {
        const double I0 = I[0], I1 = I[1];
        return (I0 - a.Rmin * (I1 - I0) * a.inv_dR) * a.pix_area;
    }
    const double x = (double)(N / 2 - c) * a.dxy;
    const double y = (double)(N / 2 - r) * a.dxy;
    const double xs = x * a.inv_cos;
    const double rho = sqrt(xs * xs + y * y);
    const double t = (rho - a.Rmin) * a.inv_dR;
    if (t >= 0.0 && t <= a.tmax) {
        int j = (int)t;
        j = j < a.Nr - 2 ? j : a.Nr - 2;
        const double f = t - (double)j;
        return ((1.0 - f) * (double)I[j] + f * (double)I[j + 1]) * a.pix_area;
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// Row pass.  Block of B rows, each a length-N real FFT done as a length-N/2
// complex FFT of z[n] = x[2n] + i x[2n+1] followed by the split
//   X[q] = (Z[q] + conj Z[L-q]) / 2 - i W_N^q (Z[q] - conj Z[L-q]) / 2.
// Output XT[q * CS + r] = (-1)^q X_r[q] for q < Q.
template <typename T, typename Cfg, bool PROFILE>
__global__ __launch_bounds__(Cfg::NT) void k_rows(const T *__restrict__ src, SweepArgs sw,
                                                  Geom g, c2<T> *__restrict__ XT) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = 2 * L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int r0 = xcd_remap(blockIdx.x, gridDim.x) * B;

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
        const c2<T> zk = lds[b * Cfg::LS + (q & (L - 1))];
        const c2<T> zc = cconj(lds[b * Cfg::LS + ((L - q) & (L - 1))]);
        const c2<T> s = cadd(zk, zc);
        const c2<T> d = cmul(wN[q], csub(zk, zc));
        c2<T> X = {half * (s.x + d.y), half * (s.y - d.x)};
        if (q & 1) X = {-X.x, -X.y};
        XT[(size_t)q * g.CS + r0 + b] = X;
    }
}

// ---------------------------------------------------------------------------
// Column pass, in place.  Block of B columns q0..q0+B-1, each a length-N
// complex FFT over the rows; output rows i in [0, 2P] hold p~ = i - P with
// sign (-1)^p~.
template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_cols(Geom g, c2<T> *__restrict__ XT) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int q0 = blockIdx.x * B;

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
        c2<T> X = lds[b * Cfg::LS + p];
        if (pt & 1) X = {-X.x, -X.y};
        XT[(size_t)q * g.CS + i] = X;
    }
}

// ---------------------------------------------------------------------------
// Sampling (Sec. 3.3, Sec. 3.4, App. D) and the chi^2 reduction (Sec. 3.1).
struct SampleArgs {
    int64_t M;
    double inv_du;             // N dxy
    double cpa, spa, cinc;     // cos PA, sin PA, cos inc
    double dRA, dDec;
    int jmax, imin, imax;      // valid stencil corners: j0 <= jmax, imin <= i0 <= imax
};

constexpr int SAMPLE_NT = 256;
constexpr int SAMPLE_PPT = 4;

struct Control {
    unsigned int counter;  // blocks done (reset by the last block)
    int flag;              // 1 once a uv point fell outside the spectrum
};

template <typename T>
__device__ __forceinline__ void sample_point(const c2<T> *__restrict__ S, const Geom &g,
                                             const SampleArgs &a, double u, double v,
                                             double &Vre, double &Vim, bool &ok) {
    double ur = u * a.cpa - v * a.spa;
    double vr = u * a.spa + v * a.cpa;
    ur *= a.cinc;
    const bool mirror = ur < 0.0;
    if (mirror) {
        ur = -ur;
        vr = -vr;
    }
    const double fu = ur * a.inv_du, fv = vr * a.inv_du;
    const double j0f = floor(fu), i0f = floor(fv);
    ok = (j0f >= 0.0) && (j0f <= (double)a.jmax) && (i0f >= (double)a.imin) &&
         (i0f <= (double)a.imax);
    if (!ok) {
        Vre = __builtin_nan("");
        Vim = __builtin_nan("");
        return;
    }
    const double s = fu - j0f, t = fv - i0f;
    const int q = (int)j0f;
    const int i = (int)i0f + g.P;
    const c2<T> *c0 = S + (size_t)q * g.CS + i;
    const c2<T> *c1 = c0 + g.CS;
    const c2<T> a00 = c0[0], a10 = c0[1], a01 = c1[0], a11 = c1[1];
    const double w00 = (1.0 - t) * (1.0 - s), w01 = (1.0 - t) * s;
    const double w10 = t * (1.0 - s), w11 = t * s;
    double br = w00 * (double)a00.x + w01 * (double)a01.x + w10 * (double)a10.x + w11 * (double)a11.x;
    double bi = w00 * (double)a00.y + w01 * (double)a01.y + w10 * (double)a10.y + w11 * (double)a11.y;
    if (mirror) bi = -bi;
    br *= a.cinc;
    bi *= a.cinc;
    const double theta = 6.283185307179586476925286766559 * (u * a.dRA + v * a.dDec);
    double sn, cs;
    sincos(theta, &sn, &cs);
    Vre = br * cs - bi * sn;
    Vim = br * sn + bi * cs;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
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

template <typename T, bool CHI2>
__global__ __launch_bounds__(SAMPLE_NT) void k_sample(
    const c2<T> *__restrict__ S, Geom g, SampleArgs a, const T *__restrict__ u,
    const T *__restrict__ v, const T *__restrict__ re, const T *__restrict__ im,
    const T *__restrict__ w, c2<T> *__restrict__ vis, double *__restrict__ partials,
    Control *ctl, double *__restrict__ chi2_out) {
    __shared__ double red[SAMPLE_NT / 64];
    __shared__ int last;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)blk * (SAMPLE_NT * SAMPLE_PPT) + threadIdx.x;
    double acc = 0.0;
    bool bad = false;
#pragma unroll
    for (int p = 0; p < SAMPLE_PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        if (k < a.M) {
            double Vre, Vim;
            bool ok;
            sample_point<T>(S, g, a, (double)u[k], (double)v[k], Vre, Vim, ok);
            bad |= !ok;
            if constexpr (CHI2) {
                const double dr = Vre - (double)re[k];
                const double di = Vim - (double)im[k];
                acc += (double)w[k] * (dr * dr + di * di);
            } else {
                vis[k] = c2<T>{(T)Vre, (T)Vim};
            }
        }
    }
    if (bad) ctl->flag = 1;
    if constexpr (CHI2) {
        const double bs = block_sum(acc, red);
        if (threadIdx.x == 0) {
            partials[blk] = bs;
            __threadfence();
            const unsigned int ticket = atomicAdd(&ctl->counter, 1u);
            last = (ticket == gridDim.x - 1);
        }
        __syncthreads();
        if (last) {
            __threadfence();
            double s = 0.0;
            for (int k = threadIdx.x; k < (int)gridDim.x; k += SAMPLE_NT) s += partials[k];
            const double tot = block_sum(s, red);
            if (threadIdx.x == 0) {
                *chi2_out = tot;
                ctl->counter = 0u;
            }
        }
    }
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

// max of u^2 + v^2 (non-negative doubles order like their bit patterns)
template <typename T>
__global__ __launch_bounds__(256) void k_rho2max(const T *__restrict__ u, const T *__restrict__ v,
                                                 int64_t M, unsigned long long *out) {
    double m = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < M;
         k += (int64_t)gridDim.x * 256) {
        const double uu = u[k], vv = v[k];
        const double r2 = uu * uu + vv * vv;
        m = r2 > m ? r2 : m;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double other = __shfl_xor(m, o, 64);
        m = other > m ? other : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_ctrl_zero(Control *ctl) {
    if (threadIdx.x == 0) {
        ctl->counter = 0u;
        ctl->flag = 0;
    }
}

}  // namespace gal
