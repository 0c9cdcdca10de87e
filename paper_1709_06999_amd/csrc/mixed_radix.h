// mixed_radix.h -- transforms for image sizes N = 2^a 3^b 5^c that are not
// powers of two.
//
// The paper advises powers of two (Sec. 3.4) but its interface takes any even
// N; these sizes run on a general path: a workgroup holds one sequence of
// length L in LDS and applies Stockham passes of radix 4, 2, 3 or 5 chosen on
// the host (MrPlan), each thread keeping its butterflies' values in registers
// between the pass's two barriers.  Twiddles come from a table of the image
// size, W[m] = exp(-2 pi i m / N), filled on the device by k_mr_twiddles at
// the head of every call (the power-of-two table does not hold these roots).
// Pass with stride NS, radix R, butterfly j in [0, L/R), k = j mod NS:
//   x_t = in[j + t L/R] W_{NS R}^{t k},  X = DFT_R(x),
//   out[(j / NS) NS R + k + t NS] = X_t,
// W_{NS R}^{t k} = W[t k (L / (NS R)) (N / L)].
#pragma once
#include "fft_block.h"

namespace gal {

constexpr int MR_MAXPASS = 16;
constexpr int MR_BPT = 4;  // butterflies per thread and pass, at most (L <= 8 NT)

struct MrPlan {
    int L;                   // transform length
    int tstride;             // N / L: W_L^x = W[x tstride]
    int np;                  // passes
    int radix[MR_MAXPASS];
};

// sin and cos of 2 pi / 3, 2 pi / 5, 4 pi / 5
#define GAL_S3 0.86602540378443864676372317075293618347140262690519
#define GAL_C5A 0.30901699437494742410229341718281905886436449558672
#define GAL_C5B -0.80901699437494742410229341718281905886436449558672
#define GAL_S5A 0.95105651629515357211643933337938214340569863412575
#define GAL_S5B 0.58778525229247312916870595463907276859765243764314

// X_k = sum_n x_n exp(-2 pi i n k / 3)
template <typename T>
__device__ __forceinline__ void dft3(c2<T> *x) {
    const c2<T> s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    const c2<T> t = {x[0].x - T(0.5) * s.x, x[0].y - T(0.5) * s.y};
    const c2<T> m = {T(GAL_S3) * d.x, T(GAL_S3) * d.y};
    x[0] = cadd(x[0], s);
    x[1] = {t.x + m.y, t.y - m.x};  // t - i m
    x[2] = {t.x - m.y, t.y + m.x};  // t + i m
}

// X_k = sum_n x_n exp(-2 pi i n k / 5): with s1 = x1 + x4, d1 = x1 - x4,
// s2 = x2 + x3, d2 = x2 - x3, A1 = x0 + c1 s1 + c2 s2, A2 = x0 + c2 s1 + c1 s2,
// B1 = s1' d1 + s2' d2, B2 = s2' d1 - s1' d2 (c_k = cos(2 pi k / 5),
// s_k' = sin(2 pi k / 5)): X1 = A1 - i B1, X4 = A1 + i B1, X2 = A2 - i B2,
// X3 = A2 + i B2.
template <typename T>
__device__ __forceinline__ void dft5(c2<T> *x) {
    const T c1 = T(GAL_C5A), c2v = T(GAL_C5B), s1 = T(GAL_S5A), s2 = T(GAL_S5B);
    const c2<T> a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    const c2<T> a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    const c2<T> A1 = {x[0].x + c1 * a1.x + c2v * a2.x, x[0].y + c1 * a1.y + c2v * a2.y};
    const c2<T> A2 = {x[0].x + c2v * a1.x + c1 * a2.x, x[0].y + c2v * a1.y + c1 * a2.y};
    const c2<T> B1 = {s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
    const c2<T> B2 = {s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
    x[0] = {x[0].x + a1.x + a2.x, x[0].y + a1.y + a2.y};
    x[1] = {A1.x + B1.y, A1.y - B1.x};
    x[4] = {A1.x - B1.y, A1.y + B1.x};
    x[2] = {A2.x + B2.y, A2.y - B2.x};
    x[3] = {A2.x - B2.y, A2.y + B2.x};
}

template <int R, typename T>
__device__ __forceinline__ void dft_r(c2<T> *x) {
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 3) dft3(x);
    else if constexpr (R == 4) dft4(x);
    else dft5(x);
}

// One Stockham pass in place on lds[0, L) (all threads of the block call it).
template <int R, int NT, typename T>
__device__ __forceinline__ void mr_pass(c2<T> *lds, const c2<T> *__restrict__ W, int L, int NS,
                                        int tstride, int tid) {
    const int LR = L / R;
    const int wstep = (L / (NS * R)) * tstride;
    c2<T> x[MR_BPT][R];
#pragma unroll
    for (int b = 0; b < MR_BPT; ++b) {
        const int j = tid + b * NT;
        if (j < LR) {
            const int k = j % NS;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const c2<T> a = lds[j + t * LR];
                x[b][t] = t == 0 ? a : cmul(a, W[t * k * wstep]);
            }
        }
    }
    __syncthreads();  // every thread has read this pass's inputs
#pragma unroll
    for (int b = 0; b < MR_BPT; ++b) {
        const int j = tid + b * NT;
        if (j < LR) {
            const int k = j % NS;
            dft_r<R>(x[b]);
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) lds[base + t * NS] = x[b][t];
        }
    }
    __syncthreads();
}

// The whole transform of lds[0, L) in natural order, followed by a barrier.
template <int NT, typename T>
__device__ __forceinline__ void mr_fft(c2<T> *lds, const c2<T> *__restrict__ W, const MrPlan &pl,
                                       int tid) {
    int NS = 1;
    for (int p = 0; p < pl.np; ++p) {
        const int R = pl.radix[p];
        if (R == 4) mr_pass<4, NT>(lds, W, pl.L, NS, pl.tstride, tid);
        else if (R == 2) mr_pass<2, NT>(lds, W, pl.L, NS, pl.tstride, tid);
        else if (R == 3) mr_pass<3, NT>(lds, W, pl.L, NS, pl.tstride, tid);
        else mr_pass<5, NT>(lds, W, pl.L, NS, pl.tstride, tid);
        NS *= R;
    }
}

// W[m] = exp(-2 pi i m / N), m in [0, N)
template <typename T>
__global__ __launch_bounds__(256) void k_mr_twiddles(c2<T> *__restrict__ W, int N) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= N) return;
    double s, c;
    sincospi(2.0 * (double)m / (double)N, &s, &c);
    W[m] = c2<T>{(T)c, (T)(-s)};
}

constexpr int MR_ROWS_NT = 512;   // image rows: L = N/2 <= 4096
constexpr int MR_COLS_NT = 1024;  // columns: L = N <= 8192
constexpr int MR_LMAX = 8192;

// Image rows, one per block (as rows_body): z[n] = x[2n] + i x[2n+1], the
// length-N/2 transform, then X[q] = (Z[q] + conj Z[L-q]) / 2
// - i W_N^q (Z[q] - conj Z[L-q]) / 2, written transposed with the shift sign:
// XT[q * CS + r] = (-1)^q X_r[q], q < Q.
template <typename T>
__global__ __launch_bounds__(MR_ROWS_NT) void k_mr_rows(const T *__restrict__ img, Geom g,
                                                        MrPlan pl, const c2<T> *__restrict__ W,
                                                        c2<T> *__restrict__ XT) {
    __shared__ c2<T> lds[MR_LMAX / 2];
    const int tid = threadIdx.x, r = blockIdx.x, L = pl.L;
    const c2<T> *row = reinterpret_cast<const c2<T> *>(img + (size_t)r * g.N);
    for (int n = tid; n < L; n += MR_ROWS_NT) lds[n] = row[n];
    __syncthreads();
    mr_fft<MR_ROWS_NT>(lds, W, pl, tid);
    const T half = T(0.5);
    for (int q = tid; q < g.Q; q += MR_ROWS_NT) {  // q <= L
        const int qa = q % L, qb = (L - qa) % L;
        const c2<T> zk = lds[qa], zc = cconj(lds[qb]);
        const c2<T> s = cadd(zk, zc);
        const c2<T> d = cmul(W[q], csub(zk, zc));
        c2<T> X = {half * (s.x + d.y), half * (s.y - d.x)};
        if (q & 1) X = {-X.x, -X.y};
        XT[(size_t)q * g.CS + r] = X;
    }
}

// Columns q < Q, one per block, in place (as cols_body): the length-N
// transform over the rows, kept rows i in [0, 2P] with p~ = i - P and the
// shift sign (-1)^p~.
template <typename T>
__global__ __launch_bounds__(MR_COLS_NT) void k_mr_cols(Geom g, MrPlan pl,
                                                        const c2<T> *__restrict__ W,
                                                        c2<T> *__restrict__ XT) {
    __shared__ c2<T> lds[MR_LMAX];
    const int tid = threadIdx.x, L = pl.L;
    c2<T> *col = XT + (size_t)blockIdx.x * g.CS;
    for (int n = tid; n < L; n += MR_COLS_NT) lds[n] = col[n];
    __syncthreads();
    mr_fft<MR_COLS_NT>(lds, W, pl, tid);
    for (int i = tid; i <= 2 * g.P; i += MR_COLS_NT) {
        const int pt = i - g.P;
        c2<T> X = lds[pt < 0 ? pt + L : pt];
        if (pt & 1) X = {-X.x, -X.y};
        col[i] = X;
    }
}

}  // namespace gal
