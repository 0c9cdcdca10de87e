// fft_block.h -- workgroup-level forward FFTs for gfx950 (wave64), FP64/FP32.
//
// A workgroup of NT threads transforms B independent sequences of length L
// (a power of two) with a Stockham auto-sort schedule: every pass takes a
// radix-R butterfly per thread from registers, exchanges through LDS, and the
// output comes out in natural order, so no bit reversal is needed.  Radix
// passes of RMAX (16 by default) come first, then one pass with the remaining
// factor.  Twiddles come from one device table holding, for every power of
// two M <= TW_MAX, the M values exp(-2 pi i m / M) at offsets [M, 2M).
//
// Pass with stride NS (product of the radices already done), radix R, for
// butterfly j in [0, L/R):  k = j mod NS,
//   x_t = in[j + t L/R] * exp(-2 pi i t k / (NS R)),  X = DFT_R(x),
//   out[(j / NS) NS R + k + t NS] = X_t.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

template <typename T>
struct alignas(2 * sizeof(T)) c2 {
    T x, y;
};

template <typename T>
__device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ c2<T> cconj(c2<T> a) { return {a.x, -a.y}; }
// a * (-i)
template <typename T>
__device__ __forceinline__ c2<T> cmul_mi(c2<T> a) { return {a.y, -a.x}; }

constexpr int TW_MAX = 16384;  // largest transform length served by the table

// cos and sin of pi/8 and sqrt(1/2)
#define GAL_C8 0.92387953251128675612818318939678828682241662586364
#define GAL_S8 0.38268343236508977172845998403039886676134456248563
#define GAL_H2 0.70710678118654752440084436210484903928483593768847

// a * exp(-2 pi i K / 16), K in [0, 16): exact forms for multiples of pi/4,
// the two constants cos(pi/8), sin(pi/8) otherwise.
template <int K, typename T>
__device__ __forceinline__ c2<T> rot16(c2<T> a) {
    constexpr int k = K & 15;
    const T c8 = T(GAL_C8), s8 = T(GAL_S8), h = T(GAL_H2);
    if constexpr (k == 0) return a;
    else if constexpr (k == 4) return {a.y, -a.x};
    else if constexpr (k == 8) return {-a.x, -a.y};
    else if constexpr (k == 12) return {-a.y, a.x};
    else if constexpr (k == 2) return {(a.x + a.y) * h, (a.y - a.x) * h};
    else if constexpr (k == 6) return {(a.y - a.x) * h, -(a.x + a.y) * h};
    else if constexpr (k == 10) return {-(a.x + a.y) * h, (a.x - a.y) * h};
    else if constexpr (k == 14) return {(a.x - a.y) * h, (a.x + a.y) * h};
    else {
        // exp(-i pi k / 8) = (cr, ci)
        constexpr int sel = k;
        T cr, ci;
        if constexpr (sel == 1) { cr = c8; ci = -s8; }
        else if constexpr (sel == 3) { cr = s8; ci = -c8; }
        else if constexpr (sel == 5) { cr = -s8; ci = -c8; }
        else if constexpr (sel == 7) { cr = -c8; ci = -s8; }
        else if constexpr (sel == 9) { cr = -c8; ci = s8; }
        else if constexpr (sel == 11) { cr = -s8; ci = c8; }
        else if constexpr (sel == 13) { cr = s8; ci = c8; }
        else { cr = c8; ci = s8; }  // 15
        return {a.x * cr - a.y * ci, a.x * ci + a.y * cr};
    }
}

template <typename T>
__device__ __forceinline__ void dft2(c2<T> *x) {
    const c2<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}

// DFT of x[0], x[S], x[2S], x[3S] in place (natural order at the same slots)
template <int S, typename T>
__device__ __forceinline__ void dft4s(c2<T> *x) {
    const c2<T> t0 = cadd(x[0], x[2 * S]);
    const c2<T> t1 = csub(x[0], x[2 * S]);
    const c2<T> t2 = cadd(x[S], x[3 * S]);
    const c2<T> t3 = cmul_mi(csub(x[S], x[3 * S]));
    x[0] = cadd(t0, t2);
    x[2 * S] = csub(t0, t2);
    x[S] = cadd(t1, t3);
    x[3 * S] = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft4(c2<T> *x) { dft4s<1>(x); }

template <typename T>
__device__ __forceinline__ void dft8(c2<T> *x) {
    // even / odd halves, then combine with exp(-2 pi i k / 8) = rot16<2k>
    c2<T> e[4] = {x[0], x[2], x[4], x[6]};
    c2<T> o[4] = {x[1], x[3], x[5], x[7]};
    dft4(e);
    dft4(o);
    o[1] = rot16<2>(o[1]);
    o[2] = rot16<4>(o[2]);
    o[3] = rot16<6>(o[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = cadd(e[k], o[k]);
        x[k + 4] = csub(e[k], o[k]);
    }
}

template <typename T>
__device__ __forceinline__ void dft16(c2<T> *x) {
    // n = 4 n1 + n2, k = k1 + 4 k2:
    // X[k1 + 4 k2] = sum_n2 W4^{n2 k2} W16^{n2 k1} sum_n1 W4^{n1 k1} x[4 n1 + n2]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4s<4>(x + n2);  // y[n2 + 4 k1]
    x[5] = rot16<1>(x[5]);
    x[6] = rot16<2>(x[6]);
    x[7] = rot16<3>(x[7]);
    x[9] = rot16<2>(x[9]);
    x[10] = rot16<4>(x[10]);
    x[11] = rot16<6>(x[11]);
    x[13] = rot16<3>(x[13]);
    x[14] = rot16<6>(x[14]);
    x[15] = rot16<9>(x[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(x + 4 * k1);  // z[4 k1 + k2] = X[k1 + 4 k2]
    c2<T> y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = x[i];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = y[4 * k1 + k2];
}

template <int R, typename T>
__device__ __forceinline__ void dftR(c2<T> *x) {
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 4) dft4(x);
    else if constexpr (R == 8) dft8(x);
    else if constexpr (R == 16) dft16(x);
    else static_assert(R == 2, "unsupported radix");
}

// radix of the pass with stride NS for a length-L transform
constexpr int pass_radix(int L, int NS, int RMAX) { return (L / NS) < RMAX ? (L / NS) : RMAX; }

// Block FFT configuration: B sequences of length L on NT threads, E values
// per thread; LDS row stride LS (complex elements).
template <typename T, int L_, int B_, int NT_, int RMAX_ = 16>
struct FFTCfg {
    static constexpr int L = L_;
    static constexpr int B = B_;
    static constexpr int NT = NT_;
    static constexpr int RMAX = RMAX_;
    static constexpr int E = B * L / NT;
    // rows padded by one element when a block holds several sequences, so
    // that lanes reading the same index of different rows hit different banks
    static constexpr int LS = (B > 1) ? L + 1 : L;
    static_assert(E >= 1 && (B * L) % NT == 0, "bad FFT configuration");
    static_assert(E % ((L < RMAX) ? L : RMAX) == 0, "E must hold whole butterflies");
    // LDS slot of element e of sequence b.  The Stockham write of the first
    // pass puts lane j at e = R j + t: a stride of R 16-byte elements that
    // sends every lane of a wave to the same banks.  XOR-ing the low three
    // bits of e (one 128-byte bank row holds 8 elements of 16 bytes) with
    // bits 4..6 gives 8 consecutive lanes 8 different bank groups in those
    // writes and keeps contiguous runs contiguous, without padding memory.
    static __device__ __forceinline__ int at(int b, int e) { return b * LS + (e ^ ((e >> 4) & 7)); }
};

// Load the inputs of the pass with stride NS from LDS into registers.
template <typename Cfg, int NS, typename T>
__device__ __forceinline__ void fft_gather(c2<T> *v, const c2<T> *lds, int tid) {
    constexpr int L = Cfg::L, NT = Cfg::NT, E = Cfg::E;
    constexpr int R = pass_radix(L, NS, Cfg::RMAX);
    constexpr int LR = L / R;
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int g = tid + i * NT;
        const int b = g / LR, j = g % LR;
#pragma unroll
        for (int t = 0; t < R; ++t) v[i * R + t] = lds[Cfg::at(b, j + t * LR)];
    }
}

// One pass with stride NS: twiddles, radix-R butterflies in registers, and
// the Stockham write of the outputs to LDS (between two barriers).
template <typename Cfg, int NS, typename T>
__device__ __forceinline__ void fft_pass(c2<T> *v, c2<T> *lds, const c2<T> *__restrict__ tw,
                                         int tid) {
    constexpr int L = Cfg::L, NT = Cfg::NT, E = Cfg::E;
    constexpr int R = pass_radix(L, NS, Cfg::RMAX);
    constexpr int LR = L / R;
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int g = tid + i * NT;
        const int j = g % LR;
        if constexpr (NS > 1) {
            const int k = j % NS;
            const c2<T> *w = tw + NS * R;  // exp(-2 pi i m / (NS R))
#pragma unroll
            for (int t = 1; t < R; ++t) v[i * R + t] = cmul(v[i * R + t], w[t * k]);
        }
        dftR<R>(v + i * R);
    }
    __syncthreads();  // every thread has read this pass's inputs
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int g = tid + i * NT;
        const int b = g / LR, j = g % LR;
        const int k = j % NS;
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int t = 0; t < R; ++t) lds[Cfg::at(b, base + t * NS)] = v[i * R + t];
    }
    __syncthreads();
}

// Run the passes from stride NS to the end; v holds this pass's inputs.  The
// natural-order result is left in LDS (element e of row b at Cfg::at(b, e)),
// followed by a barrier.  `tw` is the twiddle table.
template <typename Cfg, int NS, typename T>
__device__ __forceinline__ void fft_passes(c2<T> *v, c2<T> *lds, const c2<T> *__restrict__ tw,
                                           int tid) {
    constexpr int L = Cfg::L;
    constexpr int R = pass_radix(L, NS, Cfg::RMAX);
    fft_pass<Cfg, NS>(v, lds, tw, tid);
    if constexpr (NS * R < L) {
        fft_gather<Cfg, NS * R>(v, lds, tid);
        fft_passes<Cfg, NS * R>(v, lds, tw, tid);
    }
}

// Run the passes from stride NS up to, not including, the last one; v then
// holds the last pass's inputs (for fft_last_pass).
template <typename Cfg, int NS, typename T>
__device__ __forceinline__ void fft_passes_but_last(c2<T> *v, c2<T> *lds,
                                                    const c2<T> *__restrict__ tw, int tid) {
    constexpr int L = Cfg::L;
    constexpr int R = pass_radix(L, NS, Cfg::RMAX);
    if constexpr (NS * R < L) {
        fft_pass<Cfg, NS>(v, lds, tw, tid);
        fft_gather<Cfg, NS * R>(v, lds, tid);
        fft_passes_but_last<Cfg, NS * R>(v, lds, tw, tid);
    }
}

// stride of the last pass of a length-L transform
constexpr int last_stride(int L, int RMAX) {
    int ns = 1;
    while (ns * pass_radix(L, ns, RMAX) < L) ns *= pass_radix(L, ns, RMAX);
    return ns;
}

// The last pass in registers, for callers that keep only the first `keep`
// outputs of each sequence (natural order): out(b, e, value) is called for
// every kept element e of sequence b that this thread holds, e = j + t NS
// (t < R) for its butterflies j < NS, and the results go to their
// destination without another trip through LDS.  When keep <= NS only t = 0
// survives, which is the twiddled sum of the butterfly's inputs.
template <typename Cfg, typename T, typename Out>
__device__ __forceinline__ void fft_last_pass(c2<T> *v, const c2<T> *__restrict__ tw, int tid,
                                              int keep, Out out) {
    constexpr int L = Cfg::L, NT = Cfg::NT, E = Cfg::E;
    constexpr int NS = last_stride(L, Cfg::RMAX);
    constexpr int R = L / NS;
    static_assert(R == pass_radix(L, NS, Cfg::RMAX), "last pass");
    const c2<T> *w = tw + L;  // exp(-2 pi i m / L)
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int g = tid + i * NT;
        const int b = g / NS, j = g % NS;  // L / R = NS butterflies per sequence
        if (j >= keep) continue;
        if (NS > 1) {
#pragma unroll
            for (int t = 1; t < R; ++t) v[i * R + t] = cmul(v[i * R + t], w[t * j]);
        }
        if (keep <= NS) {
            c2<T> s = v[i * R];
#pragma unroll
            for (int t = 1; t < R; ++t) s = cadd(s, v[i * R + t]);
            out(b, j, s);
        } else {
            dftR<R>(v + i * R);
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (j + t * NS < keep) out(b, j + t * NS, v[i * R + t]);
        }
    }
}

}  // namespace gal
