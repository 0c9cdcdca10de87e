// adjoint.h -- gradient of chi^2 with respect to the image pixels and to the
// profile values (the paper gives no gradient; this is the exact transpose of
// the forward path, written for the same data layouts).
//
// chi^2 = sum_k w_k |R_k|^2, R_k = Vobs_k - V_k, and V_k is linear in the
// image, so d chi^2 / d img = -2 sum_k w_k Re(conj(R_k) dV_k / d img).
//
// General image (complex half spectrum S, node n = (q, p~)):
//   V_k = cinc e^{i theta_k} F_k(sum_n beta_kn S_n), F_k = conj for mirrored
//   points, and S_n = sum_x img[x] E_n(x), E_n = exp(-2 pi i (p~ (r-N/2) +
//   q (c-N/2)) / N).  Then
//     d chi^2 / d img[x] = -2 Re sum_n A_n E_n(x),
//     A_n = sum_k w_k cinc beta_kn a_k,  a_k = conj(R_k) e^{i theta_k}
//   (mirrored: a_k = R_k e^{-i theta_k}).  A is scattered onto the stored
//   nodes, transformed along p for every kept column (length-N FFT, all rows
//   r) and then along q for every row: Re of a length-N FFT of a sequence
//   that is zero beyond q >= Q, done two rows at a time through its Hermitian
//   extension (whose transform is real).
//
// Swept profile (real spectrum S_R[p][q], p >= 0, node p~ read at |p~|):
//   along even images G[p][q] = sum img cos(phi_p(r)) cos(phi_q(c)), so
//     d chi^2 / d img[r][c] (even part) = -2 sum_{p,q} A_R[p][q] cos phi_p(r) cos phi_q(c),
//     A_R[p][q] = sum_k w_k beta_kn Re(conj(R_k) e^{i theta_k}) over nodes at (|p~|, q),
//   two real cosine transforms (even extensions packed two at a time), on the
//   quadrant r, c in [0, N/2] only; then the transpose of the sweep sums the
//   pixel gradient into the profile bins (each quadrant pixel stands for its
//   mirrors: weight m(r) m(c), m = 1 on the rows/columns 0 and N/2, else 2).
#pragma once
#include "kernels.h"

namespace gal {

// Zero [p, p + pb) and [q, q + qb) (16-byte aligned, sizes multiples of 8
// bytes) with 16-byte stores; the grid is sized to the ranges (zero_grid).
__global__ __launch_bounds__(256) void k_zero16(void *__restrict__ p, int64_t pb,
                                                void *__restrict__ q, int64_t qb) {
    const int64_t n1 = pb >> 4, n2 = qb >> 4;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n1 + n2; i += stride) {
        uint4 *d = i < n1 ? (uint4 *)p + i : (uint4 *)q + (i - n1);
        *d = make_uint4(0u, 0u, 0u, 0u);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // an 8-byte tail of either range
        if (pb & 8) ((unsigned long long *)p)[(pb >> 3) - 1] = 0ull;
        if (qb & 8) ((unsigned long long *)q)[(qb >> 3) - 1] = 0ull;
    }
}

inline unsigned zero_grid(int64_t bytes) {
    const int64_t b = (bytes / 16 + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// ---- block scatter through an LDS tile --------------------------------------
// Each point adds hv * wa * ws to the four nodes of its stencil, node (q, i)
// at flat index q * CS + i (times NV components: 1 real, 2 complex), with
// wa = 1 - a at i and a at i + 1, ws = 1 - s at q and s at q + 1.  The points
// of one sampling block are consecutive in the locality order of datasets,
// a compact patch of the uv plane, so their nodes span a small box.  The box
// is covered by windows of whole q-rows that fit an LDS tile; per window the
// points add into the tile (one LDS atomic per node value) and the tile is
// added to the grid row by row with one global atomic per touched value.
// That turns scattered global atomics into coalesced ones, and in dense uv
// cores, where thousands of points share a node, into a few.  A box larger
// than SCAT_WINDOWS tiles (sparse points spread thin, where clearing and
// scanning the box would cost more than the atomics it saves) falls back to
// direct global atomics.
constexpr int SCAT_TILE = 4096;  // doubles of LDS per block
constexpr int SCAT_WINDOWS = 2;

template <int NV>
struct PointAdd {
    int q, i;         // q < 0: nothing to add
    double hv[NV];
    double a, s;
};

// Called by every thread of the block (it synchronises); tile: SCAT_TILE
// doubles of LDS, box: 4 * (blockDim.x / 64) ints of LDS.
template <typename T, int NV, int NP>
__device__ __forceinline__ void block_scatter(T *__restrict__ A, int CS, const PointAdd<NV> (&pa)[NP],
                                              double *tile, int *box) {
    constexpr int BIG = 0x3fffffff;
    int qlo = BIG, qhi = -BIG, ilo = BIG, ihi = -BIG;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (pa[p].q < 0) continue;
        qlo = min(qlo, pa[p].q);
        qhi = max(qhi, pa[p].q);
        ilo = min(ilo, pa[p].i);
        ihi = max(ihi, pa[p].i);
    }
    qlo = wave_min(qlo);
    qhi = wave_max(qhi);
    ilo = wave_min(ilo);
    ihi = wave_max(ihi);
    const int nw = (int)(blockDim.x >> 6), wid = (int)(threadIdx.x >> 6);
    __syncthreads();  // the previous call's readers of box and tile are done
    if ((threadIdx.x & 63) == 0) {
        box[4 * wid] = qlo;
        box[4 * wid + 1] = qhi;
        box[4 * wid + 2] = ilo;
        box[4 * wid + 3] = ihi;
    }
    __syncthreads();
    for (int k = 0; k < nw; ++k) {
        qlo = min(qlo, box[4 * k]);
        qhi = max(qhi, box[4 * k + 1]);
        ilo = min(ilo, box[4 * k + 2]);
        ihi = max(ihi, box[4 * k + 3]);
    }
    // the same in every lane of the block: scalar from here on
    qlo = __builtin_amdgcn_readfirstlane(qlo);
    qhi = __builtin_amdgcn_readfirstlane(qhi);
    ilo = __builtin_amdgcn_readfirstlane(ilo);
    ihi = __builtin_amdgcn_readfirstlane(ihi);
    if (qlo > qhi) return;  // no point of the block adds anything (uniform)
    const int TQ = qhi - qlo + 2, TI = ihi - ilo + 2;
    const int SQ = SCAT_TILE / (TI * NV);  // q-rows per window
    if (SQ < 1 || TQ * TI * NV > SCAT_WINDOWS * SCAT_TILE) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (pa[p].q < 0) continue;
            const size_t n = (size_t)pa[p].q * CS + pa[p].i;
            const double wa[2] = {1.0 - pa[p].a, pa[p].a}, ws[2] = {1.0 - pa[p].s, pa[p].s};
#pragma unroll
            for (int dq = 0; dq < 2; ++dq)
#pragma unroll
                for (int di = 0; di < 2; ++di)
#pragma unroll
                    for (int c = 0; c < NV; ++c)
                        atomicAdd(&A[(n + (size_t)dq * CS + di) * NV + c],
                                  (T)(pa[p].hv[c] * wa[di] * ws[dq]));
        }
        return;
    }
    // node values of point 0 with the later points of the same stencil folded
    // in (dense uv cores: fewer conflicting adds); `own` marks the others
    double acc[4][NV];
    bool own[NP];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[n][c] = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        own[p] = false;
        if (pa[p].q < 0) continue;
        if (p > 0 && (pa[p].q != pa[0].q || pa[p].i != pa[0].i)) {
            own[p] = true;
            continue;
        }
        const double wa[2] = {1.0 - pa[p].a, pa[p].a}, ws[2] = {1.0 - pa[p].s, pa[p].s};
#pragma unroll
        for (int dq = 0; dq < 2; ++dq)
#pragma unroll
            for (int di = 0; di < 2; ++di)
#pragma unroll
                for (int c = 0; c < NV; ++c) acc[2 * dq + di][c] += pa[p].hv[c] * wa[di] * ws[dq];
    }
    // flat index -> (row, column) of a window: exact in float for indices
    // below 2^12 (the quotient stays >= 0.5/TI from an integer, far above the
    // float rounding of k/TI)
    const float inv = 1.0f / (float)TI;
    for (int w0 = qlo; w0 < qlo + TQ; w0 += SQ) {
        const int w1 = min(w0 + SQ, qlo + TQ);  // q-rows [w0, w1) of this window
        const int nk = (w1 - w0) * TI;
        for (int k = threadIdx.x; k < nk * NV; k += blockDim.x) tile[k] = 0.0;
        __syncthreads();
        if (pa[0].q >= 0) {
#pragma unroll
            for (int dq = 0; dq < 2; ++dq) {
                const int qn = pa[0].q + dq;
                if (qn < w0 || qn >= w1) continue;
#pragma unroll
                for (int di = 0; di < 2; ++di)
#pragma unroll
                    for (int c = 0; c < NV; ++c)
                        atomicAdd(&tile[((qn - w0) * TI + pa[0].i + di - ilo) * NV + c],
                                  acc[2 * dq + di][c]);
            }
        }
#pragma unroll
        for (int p = 1; p < NP; ++p) {
            if (!own[p]) continue;
            const double wa[2] = {1.0 - pa[p].a, pa[p].a}, ws[2] = {1.0 - pa[p].s, pa[p].s};
#pragma unroll
            for (int dq = 0; dq < 2; ++dq) {
                const int qn = pa[p].q + dq;
                if (qn < w0 || qn >= w1) continue;
#pragma unroll
                for (int di = 0; di < 2; ++di)
#pragma unroll
                    for (int c = 0; c < NV; ++c)
                        atomicAdd(&tile[((qn - w0) * TI + pa[p].i + di - ilo) * NV + c],
                                  pa[p].hv[c] * wa[di] * ws[dq]);
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nk; k += blockDim.x) {
            const int dq = (int)(((float)k + 0.5f) * inv), di = k - dq * TI;
            const size_t n = (size_t)(w0 + dq) * CS + (ilo + di);
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double v = tile[k * NV + c];
                if (v != 0.0) atomicAdd(&A[n * NV + c], (T)v);
            }
        }
        __syncthreads();  // the flush has read the tile before it is cleared
    }
}

// The residual R_k = Vobs_k - V_k of one sampled point as node additions.
// Real spectrum (swept profile): hv = w cinc Re(conj(R) e^{i theta}) on the
// even-form stencil (stored rows i and i + 1 with weights 1 - t and t).
template <typename T>
__device__ __forceinline__ PointAdd<1> point_add_real(const StencilE<T> &st, double h) {
    PointAdd<1> r;
    r.q = st.q;
    r.i = st.i;
    r.hv[0] = h;
    r.a = st.t;
    r.s = st.s;
    return r;
}

// Complex half spectrum (image): hv = w cinc a_k, a_k = conj(R) e^{i theta}
// (direct) or R e^{-i theta} (mirrored).
template <typename T>
__device__ __forceinline__ PointAdd<2> point_add_cplx(const Stencil<T> &st, double h, double R0,
                                                      double R1, double sn, double cs) {
    PointAdd<2> r;
    r.q = st.q;
    r.i = st.i;
    r.hv[0] = h * (R0 * cs + R1 * sn);
    r.hv[1] = h * (st.mirror ? (R1 * cs - R0 * sn) : (R0 * sn - R1 * cs));
    r.a = st.t;
    r.s = st.s;
    return r;
}

// ---- sampling + scatter ----------------------------------------------------
// Forward sample of every point (chi^2 partials as in k_sample*), then the
// residuals added to the adjoint grid A (same layout as the spectrum).
template <typename T, bool REAL>
__global__ __launch_bounds__(SAMPLE_NT) void k_sample_scatter(
    const T *__restrict__ S, T *__restrict__ A, Geom g, SampleArgs a, const T *__restrict__ u,
    const T *__restrict__ v, const T *__restrict__ re, const T *__restrict__ im,
    const T *__restrict__ w, double *__restrict__ partials, Control *ctl) {
    constexpr int NV = REAL ? 1 : 2;
    __shared__ double red[SAMPLE_NT / 64];
    __shared__ double tile[SCAT_TILE];
    __shared__ int box[4 * (SAMPLE_NT / 64)];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    if (a.M == 0) {  // an empty dataset: one block, nothing to read
        if (threadIdx.x == 0) partials[blk] = 0.0;
        return;
    }
    // each thread takes SAMPLE_PPT consecutive points: neighbours in the
    // locality order of datasets, which in dense regions share a stencil.
    // No branch per point: a point past M re-reads point M - 1 and adds
    // nothing, so the loads and gathers of all points can be in flight
    // together.
    const int64_t base = (int64_t)blk * (SAMPLE_NT * SAMPLE_PPT) + threadIdx.x * SAMPLE_PPT;
    double acc = 0.0;
    bool bad = false;
    PointAdd<NV> pa[SAMPLE_PPT];
#pragma unroll
    for (int p = 0; p < SAMPLE_PPT; ++p) {
        pa[p].q = -1;
        const int64_t k = base + p;
        const bool in = k < a.M;
        const int64_t kk = in ? k : a.M - 1;
        const double uu = u[kk], vv = v[kk];
        const double ov = re[kk], oi = im[kk], wk = w[kk];
        double sn, cs;
        phase_of(a, uu, vv, sn, cs);
        if constexpr (REAL) {
            // an off-grid stencil points at valid nodes; its value is discarded
            const StencilE<T> st = locate_e<T>(g, a, uu, vv);
            double x0, x1, y0, y1;
            nodes_e<T>(S, st, g.CS, x0, x1, y0, y1);
            const double b = bilerp(x0, y0, x1, y1, st.s, st.t);
            const double Vre = b * cs, Vim = b * sn;  // cos(inc) = 1 on real spectra
            const double rr = ov - Vre, ri = oi - Vim;
            bad |= in && !st.ok;
            acc += (in && st.ok) ? wk * (rr * rr + ri * ri) : (in ? __builtin_nan("") : 0.0);
            // Re(conj(R) e^{i theta}) = rr cs + ri sn
            if (in && st.ok) pa[p] = point_add_real<T>(st, wk * (rr * cs + ri * sn));
        } else {
            const c2<T> *Sc = (const c2<T> *)S;
            const Stencil<T> st = locate<T>(Sc, g, a, uu, vv);
            const c2<T> n00 = st.c0[0], n10 = st.c0[1], n01 = st.c0[g.CS], n11 = st.c0[g.CS + 1];
            const double s = st.s, t = st.t;
            const double w00 = (1.0 - t) * (1.0 - s), w01 = (1.0 - t) * s;
            const double w10 = t * (1.0 - s), w11 = t * s;
            double br = w00 * n00.x + w01 * n01.x + w10 * n10.x + w11 * n11.x;
            double bi = w00 * n00.y + w01 * n01.y + w10 * n10.y + w11 * n11.y;
            if (st.mirror) bi = -bi;
            br *= a.cinc;
            bi *= a.cinc;
            const double Vre = br * cs - bi * sn, Vim = br * sn + bi * cs;
            const double rr = ov - Vre, ri = oi - Vim;
            bad |= in && !st.ok;
            acc += (in && st.ok) ? wk * (rr * rr + ri * ri) : (in ? __builtin_nan("") : 0.0);
            if (in && st.ok) pa[p] = point_add_cplx<T>(st, wk * a.cinc, rr, ri, sn, cs);
        }
    }
    if (bad) atomicOr(&ctl->flag, STATUS_UV);
    block_scatter<T, NV, SAMPLE_PPT>(A, g.CS, pa, tile, box);
    const double bs = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blk] = bs;
}

// ---- general image: columns ------------------------------------------------
// Column q of A (rows i = p~ + P, i in [0, 2P]) -> H[r][q] = sum_p~ A (-1)^p~
// exp(-2 pi i p~ r / N) for all r in [0, N), written in place (stride CS).
template <typename T, typename Cfg>
__device__ __forceinline__ void adj_cols_body(const Geom &g, c2<T> *__restrict__ A, int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = L;
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
            const int n = j + t * LR;             // frequency index p = p~ mod N
            const int pt = n < N / 2 ? n : n - N; // p~ in [-N/2, N/2)
            c2<T> x{T(0), T(0)};
            if (q < g.Q) {
                if (pt >= -g.P && pt <= g.P) x = A[(size_t)q * g.CS + pt + g.P];
                if (pt == -N / 2 && g.P >= N / 2) {  // p~ = +N/2 is the same frequency
                    const c2<T> y = A[(size_t)q * g.CS + N / 2 + g.P];
                    x = cadd(x, y);
                }
                if (pt & 1) x = {-x.x, -x.y};
            }
            v[i * R0 + t] = x;
        }
    }
    fft_passes<Cfg, 1>(v, lds, twiddles<T>(), tid);
    for (int idx = tid; idx < N * B; idx += NT) {
        const int b = idx / N, r = idx % N;
        const int q = q0 + b;
        if (q >= g.Q) continue;
        A[(size_t)q * g.CS + r] = lds[Cfg::at(b, r)];
    }
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_adj_cols(Geom g, c2<T> *__restrict__ A) {
    adj_cols_body<T, Cfg>(g, A, blockIdx.x);
}

// ---- general image: rows ---------------------------------------------------
// Rows 2m, 2m+1: h_r[q] = (-1)^q H[r][q] (q < Q), Hermitian extension x_r
// (x[0] = Re h[0], x[q] = h[q]/2, x[N-q] = conj(h[q])/2, x[N/2] = Re h[N/2]),
// z = x_{2m} + i x_{2m+1}; grad[r][c] = -2 Re / Im of FFT(z)[c].
template <typename T, typename Cfg>
__device__ __forceinline__ void adj_rows_body(const Geom &g, const c2<T> *__restrict__ H,
                                              T *__restrict__ grad, int blk, bool nan_out = false) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int m0 = blk * B;
    const T half = T(0.5);
    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
        const int r = 2 * (m0 + b);
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            c2<T> z{T(0), T(0)};
            const int qq = n <= N / 2 ? n : N - n;
            if (r < N && qq < g.Q) {
                c2<T> h1 = H[(size_t)qq * g.CS + r], h2 = H[(size_t)qq * g.CS + r + 1];
                if (qq & 1) {
                    h1 = {-h1.x, -h1.y};
                    h2 = {-h2.x, -h2.y};
                }
                if (qq == 0 || qq == N / 2) {
                    z = {h1.x, h2.x};
                } else if (n < N / 2) {  // h1/2 + i h2/2
                    z = {half * (h1.x - h2.y), half * (h1.y + h2.x)};
                } else {                 // conj(h1)/2 + i conj(h2)/2
                    z = {half * (h1.x + h2.y), half * (h2.x - h1.y)};
                }
            }
            v[i * R0 + t] = z;
        }
    }
    fft_passes<Cfg, 1>(v, lds, twiddles<T>(), tid);
    for (int idx = tid; idx < 2 * B * N; idx += NT) {
        const int rb = idx / N, c = idx % N;
        const int r = 2 * m0 + rb;
        if (r >= N) continue;
        const c2<T> z = lds[Cfg::at(rb >> 1, c)];
        const T gv = T(-2) * ((rb & 1) ? z.y : z.x);
        grad[(size_t)r * N + c] = nan_out ? T(__builtin_nan("")) : gv;
    }
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_adj_rows(Geom g, const c2<T> *__restrict__ H,
                                                      T *__restrict__ grad) {
    adj_rows_body<T, Cfg>(g, H, grad, xcd_remap(blockIdx.x, gridDim.x));
}

// ---- swept profile: columns -------------------------------------------------
// Column pair (2m, 2m+1) of A_R (p in [0, P]): even extension over p of
// (-1)^p A_R[p][q] halved off p = 0 (and p = N/2), packed re/im; its
// transform is H[r][q] = sum_p A_R[p][q] (-1)^p cos(2 pi p r / N), kept for
// r in [0, N/2] in place.
template <typename T, typename Cfg>
__device__ __forceinline__ void adj_cols_sym_body(const Geom &g, int Qe, T *__restrict__ A,
                                                  int blk) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int N = L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    const int tid = threadIdx.x;
    const int m0 = blk * B;
    if (2 * m0 >= Qe) return;
    const T half = T(0.5);
    c2<T> v[E];
#pragma unroll
    for (int i = 0; i < E / R0; ++i) {
        const int gi = tid + i * NT;
        const int b = gi / LR, j = gi % LR;
        const int q = 2 * (m0 + b);
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int n = j + t * LR;
            const int pp = n <= N / 2 ? n : N - n;
            c2<T> x{T(0), T(0)};
            if (q < Qe && pp <= g.P) {
                x = {A[(size_t)q * g.CS + pp], A[(size_t)(q + 1) * g.CS + pp]};
                if (pp & 1) x = {-x.x, -x.y};
                if (pp != 0 && pp != N / 2) x = {half * x.x, half * x.y};
            }
            v[i * R0 + t] = x;
        }
    }
    fft_passes<Cfg, 1>(v, lds, twiddles<T>(), tid);
    constexpr int NH = N / 2 + 1;
    for (int idx = tid; idx < NH * 2 * B; idx += NT) {
        const int cb = idx / NH, r = idx % NH;
        const int q = 2 * m0 + cb;
        if (q >= Qe) continue;
        const c2<T> z = lds[Cfg::at(cb >> 1, r)];
        A[(size_t)q * g.CS + r] = (cb & 1) ? z.y : z.x;
    }
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_adj_cols_sym(Geom g, int Qe, T *__restrict__ A) {
    adj_cols_sym_body<T, Cfg>(g, Qe, A, blockIdx.x);
}

// ---- swept profile: rows and the transposed sweep ----------------------------
// Quadrant rows r = 2m, 2m+1 (<= N/2): g_r[c] = -2 sum_q (-1)^q H[r][q]
// cos(2 pi q c / N) over the even extension in q, c in [0, N/2] -- the
// transform of an even sequence, taken at half length by even_transform with
// x[0] = H[r][0], x[q] = (-1)^q H[r][q] / 2 for 0 < q < N/2 (the extension
// counts those twice) and x[N/2] = (-1)^(N/2) H[r][N/2].  Each pixel then
// adds m(r) m(c) g dxy^2 (1 - f) to bin j and ... f to bin j+1 (centre pixel:
// (1 + Rmin/dR) to bin 0 and -Rmin/dR to bin 1) in an LDS histogram, flushed
// with one atomic per touched bin into gI, one of GI_COPIES copies of the bin
// accumulator (the kernels pick it by block index): the outer bins are
// reached by almost every row pair, and same-address atomics serialise, so
// the copies split those chains; k_sum_bins adds the copies afterwards.
// A block takes ppb consecutive
// groups of B row pairs and flushes its histogram once: a row pair touches
// thousands of bins, so the flush's global atomics, not the transform, bound
// a pass with one group per block.  Cfg is the half-length shape (L = N/2),
// as for rows_even_body.
constexpr int GI_COPIES = 16;
template <typename T, typename Cfg>
__device__ __forceinline__ void adj_rows_sym_body(const Geom &g, const T *__restrict__ H,
                                                  const SweepArgs &sw, double *__restrict__ gI,
                                                  double *hist, int blk, int ppb) {
    constexpr int L = Cfg::L, B = Cfg::B, NT = Cfg::NT, E = Cfg::E;
    constexpr int h = L, N = 2 * L;
    constexpr int R0 = pass_radix(L, 1, Cfg::RMAX);
    constexpr int LR = L / R0;
    __shared__ c2<T> lds[B * Cfg::LS];
    __shared__ c2<T> xh[B];
    __shared__ c2<double> part[B * LR];
    __shared__ int jlo_s, jhi_s;
    const int tid = threadIdx.x;
    const int Qr = g.Q;  // kept columns (<= N/2 + 1)
    const T half = T(0.5);
    // x[q] of rows r (in .x) and r + 1 (in .y); row N/2 + 1 is not kept
    auto load = [&](int r, int q) {
        c2<T> x{T(0), T(0)};
        if (r <= N / 2 && q < Qr) {
            const T *src = H + (size_t)q * g.CS + r;
            x = (r + 1 <= N / 2) ? *reinterpret_cast<const c2<T> *>(src) : c2<T>{src[0], T(0)};
            if (q & 1) x = {-x.x, -x.y};
        }
        return x;
    };
    for (int k = tid; k < sw.Nr; k += NT) hist[k] = 0.0;
    if (tid == 0) {
        jlo_s = sw.Nr;
        jhi_s = -1;
    }
    int jlo = sw.Nr, jhi = -1;
    // pixel (r, c) with the value X of the transform
    auto pixel = [&](int r, int c, double X) {
        const double mult = ((r == 0 || r == N / 2) ? 1.0 : 2.0) * ((c == 0 || c == N / 2) ? 1.0 : 2.0);
        const double gw = -2.0 * X * mult * sw.pix_area;
        if (r == N / 2 && c == N / 2) {
            atomicAdd(&hist[0], gw * (1.0 - sw.t0));
            atomicAdd(&hist[1], gw * sw.t0);
            jlo = 0;
            jhi = jhi > 1 ? jhi : 1;
            return;
        }
        const double xs = (double)(N / 2 - c) * sw.dxs;  // as sweep_pixel
        const double y = (double)(N / 2 - r) * sw.dxy;
        const double rho = sqrt_pos(fma(xs, xs, y * y));
        const double tt = sweep_t(rho, sw);
        if (tt >= 0.0 && tt <= sw.tmax) {
            int j = (int)tt;
            j = j < sw.Nr - 2 ? j : sw.Nr - 2;
            const double f = tt - (double)j;
            atomicAdd(&hist[j], gw * (1.0 - f));
            atomicAdd(&hist[j + 1], gw * f);
            jlo = j < jlo ? j : jlo;
            jhi = j + 1 > jhi ? j + 1 : jhi;
        }
    };
    static_assert(B * h == E * NT, "staging: E values per thread");
    for (int i = 0; i < ppb; ++i) {
        const int m0 = (blk * ppb + i) * B;
        if (2 * m0 > N / 2) break;  // the same for the whole block
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int idx = tid + k * NT;
            const int b = idx / h, q = idx % h;
            c2<T> x = load(2 * (m0 + b), q);
            if (q != 0) x = {half * x.x, half * x.y};
            lds[Cfg::at(b, q)] = x;
        }
        if (tid < B) xh[tid] = load(2 * (m0 + tid), h);
        __syncthreads();
        // m in [0, h/2]: columns 2m and 2m + 1 (<= h)
        even_transform<T, Cfg, B == 1>(
            lds, xh, part, tid, h / 2 + 1, [&](int b) { return 2 * (m0 + b) <= N / 2; },
            [&](int b, int m, c2<T> ev, c2<T> od) {
                const int r = 2 * (m0 + b);
                const bool two = r + 1 <= N / 2;
                pixel(r, 2 * m, (double)ev.x);
                if (two) pixel(r + 1, 2 * m, (double)ev.y);
                if (2 * m + 1 <= h) {
                    pixel(r, 2 * m + 1, -(double)od.x);
                    if (two) pixel(r + 1, 2 * m + 1, -(double)od.y);
                }
            });
        __syncthreads();  // before the next group is staged over this one
    }
    jlo = wave_min(jlo);  // one LDS atomic per wave instead of one per thread
    jhi = wave_max(jhi);
    if ((tid & 63) == 0) {
        atomicMin(&jlo_s, jlo);
        atomicMax(&jhi_s, jhi);
    }
    __syncthreads();
    for (int k = jlo_s + tid; k <= jhi_s; k += NT) {
        const double hv = hist[k];
        if (hv != 0.0) atomicAdd(&gI[k], hv);
    }
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_adj_rows_sym(Geom g, const T *__restrict__ H,
                                                          SweepArgs sw, double *__restrict__ gI,
                                                          int ppb) {
    extern __shared__ double hist[];
    adj_rows_sym_body<T, Cfg>(g, H, sw, gI + (size_t)(blockIdx.x % GI_COPIES) * sw.Nr, hist,
                              xcd_remap(blockIdx.x, gridDim.x), ppb);
}

// profile gradient: the sum of the accumulator copies, in the array type
template <typename T>
__device__ __forceinline__ void sum_bins(const double *__restrict__ copies, int n, T *out, int i) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < GI_COPIES; ++c) s += copies[(size_t)c * n + i];
    out[i] = (T)s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_sum_bins(const double *__restrict__ copies, int n,
                                                  T *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) sum_bins<T>(copies, n, out, i);
}

}  // namespace gal
