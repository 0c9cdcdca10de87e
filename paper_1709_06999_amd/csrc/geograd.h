// geograd.h -- chi^2 and its derivatives with respect to the geometry: PA,
// the offsets dRA, dDec and the inclination (not in the paper).
//
// With R = Vobs - V, d chi^2 / d a = -2 sum_k w_k Re(conj(R_k) dV_k / d a):
//  - offsets: V = V^ exp(i theta), theta = 2 pi (u dRA + v dDec), so
//    dV/d dRA = 2 pi i u V and dV/d dDec = 2 pi i v V;
//  - PA moves the sampling point: u' = u cos PA - v sin PA, v' = u sin PA +
//    v cos PA give du'/dPA = -v', dv'/dPA = u'; the grid coordinates are
//    fu = m u' cinc / du, fv = m v' / du (m = -1 for a mirrored point), and
//    the bilinear value B(s, t) of the stencil has
//      dB/ds = (1-t)(B(q+1, i) - B(q, i)) + t (B(q+1, i+1) - B(q, i+1)),
//      dB/dt = (1-s)(B(q, i+1) - B(q, i)) + s (B(q+1, i+1) - B(q+1, i));
//  - inclination of an image (inc of *Image, the u' cos(inc) deprojection
//    and flux factor): V^ = cinc conj_m(B), dfu/dinc = -m u' sin(inc) / du;
//  - inclination of a swept profile: the image itself depends on inc, so
//    dV/dinc samples, at the same stencil, the spectrum of the image
//    d img / d inc (sweep_pixel_dinc) transformed by the same passes.
// The derivative of the bilinear interpolant is the one inside the cell
// (it jumps across cell edges).
#pragma once
#include "kernels.h"

namespace gal {

constexpr int GEO_N = 5;  // chi^2, d/dPA, d/d dRA, d/d dDec, d/d inc

template <typename T, bool REAL>
__global__ __launch_bounds__(SAMPLE_NT) void k_sample_geo(
    const T *__restrict__ S, const T *__restrict__ St, Geom g, SampleArgs a, double sinc,
    const T *__restrict__ u, const T *__restrict__ v, const T *__restrict__ re,
    const T *__restrict__ im, const T *__restrict__ w, double *__restrict__ partials,
    Control *ctl) {
    __shared__ double red[SAMPLE_NT / 64];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)blk * (SAMPLE_NT * SAMPLE_PPT) + threadIdx.x;
    double acc[GEO_N] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool bad = false;
#pragma unroll
    for (int p = 0; p < SAMPLE_PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        if (k >= a.M) continue;
        const double uu = u[k], vv = v[k];
        double sn, cs;
        phase_of(a, uu, vv, sn, cs);
        const double up = uu * a.cpa - vv * a.spa, vp = uu * a.spa + vv * a.cpa;
        double Br, Bi = 0.0, Bsr, Bsi = 0.0, Btr, Bti = 0.0, Ir, Ii = 0.0;
        double s, t;
        bool mirror;
        if constexpr (REAL) {
            const StencilR<T> st = locate_r<T>(S, g, a, uu, vv);
            if (!st.ok) {
                bad = true;
                acc[0] = __builtin_nan("");
                continue;
            }
            mirror = uu * a.cpa_du - vv * a.spa_du < 0.0;  // the sign test of locate_r
            s = st.s;
            t = st.t;
            // node values at (q, p~0), (q, p~0+1), (q+1, p~0), (q+1, p~0+1)
            const T x0 = st.c0[0], x1 = st.c0[1], y0 = st.c0[g.CS], y1 = st.c0[g.CS + 1];
            const double a00 = st.swap ? x1 : x0, a10 = st.swap ? x0 : x1;
            const double a01 = st.swap ? y1 : y0, a11 = st.swap ? y0 : y1;
            Br = (1.0 - t) * ((1.0 - s) * a00 + s * a01) + t * ((1.0 - s) * a10 + s * a11);
            Bsr = (1.0 - t) * (a01 - a00) + t * (a11 - a10);
            Btr = (1.0 - s) * (a10 - a00) + s * (a11 - a01);
            const T *c1 = St + (st.c0 - S);  // the tangent spectrum at the same nodes
            const T z0 = c1[0], z1 = c1[1], z2 = c1[g.CS], z3 = c1[g.CS + 1];
            const double e00 = st.swap ? z1 : z0, e10 = st.swap ? z0 : z1;
            const double e01 = st.swap ? z3 : z2, e11 = st.swap ? z2 : z3;
            Ir = (1.0 - t) * ((1.0 - s) * e00 + s * e01) + t * ((1.0 - s) * e10 + s * e11);
        } else {
            const c2<T> *Sc = (const c2<T> *)S;
            const Stencil<T> st = locate<T>(Sc, g, a, uu, vv);
            if (!st.ok) {
                bad = true;
                acc[0] = __builtin_nan("");
                continue;
            }
            mirror = st.mirror;
            s = st.s;
            t = st.t;
            // (q, i), (q, i+1), (q+1, i), (q+1, i+1)
            const c2<T> n00 = st.c0[0], n10 = st.c0[1], n01 = st.c0[g.CS], n11 = st.c0[g.CS + 1];
            Br = (1.0 - t) * ((1.0 - s) * n00.x + s * n01.x) + t * ((1.0 - s) * n10.x + s * n11.x);
            Bi = (1.0 - t) * ((1.0 - s) * n00.y + s * n01.y) + t * ((1.0 - s) * n10.y + s * n11.y);
            Bsr = (1.0 - t) * ((double)n01.x - n00.x) + t * ((double)n11.x - n10.x);
            Bsi = (1.0 - t) * ((double)n01.y - n00.y) + t * ((double)n11.y - n10.y);
            Btr = (1.0 - s) * ((double)n10.x - n00.x) + s * ((double)n11.x - n01.x);
            Bti = (1.0 - s) * ((double)n10.y - n00.y) + s * ((double)n11.y - n01.y);
            if (mirror) {
                Bi = -Bi;
                Bsi = -Bsi;
                Bti = -Bti;
            }
            const double dfu_dinc = (mirror ? up : -up) * sinc * a.inv_du;
            Ir = -sinc * Br + a.cinc * Bsr * dfu_dinc;
            Ii = -sinc * Bi + a.cinc * Bsi * dfu_dinc;
        }
        const double m = mirror ? -1.0 : 1.0;
        const double dfu_dpa = m * a.cinc * (-vp) * a.inv_du, dfv_dpa = m * up * a.inv_du;
        const double Vr = a.cinc * Br, Vi = a.cinc * Bi;
        const double Pr = a.cinc * (Bsr * dfu_dpa + Btr * dfv_dpa);
        const double Pi = a.cinc * (Bsi * dfu_dpa + Bti * dfv_dpa);
        const double VVr = Vr * cs - Vi * sn, VVi = Vr * sn + Vi * cs;
        const double Rr = (double)re[k] - VVr, Ri = (double)im[k] - VVi;
        const double ww = (double)w[k];
        const double Pr2 = Pr * cs - Pi * sn, Pi2 = Pr * sn + Pi * cs;
        const double Ir2 = Ir * cs - Ii * sn, Ii2 = Ir * sn + Ii * cs;
        // Re(conj(R) i X) = -Im(conj(R) X) = -(Rr Xi - Ri Xr)
        const double imRV = Rr * VVi - Ri * VVr;
        const double two_pi = 6.283185307179586;
        acc[0] += ww * (Rr * Rr + Ri * Ri);
        acc[1] += -2.0 * ww * (Rr * Pr2 + Ri * Pi2);
        acc[2] += 2.0 * ww * two_pi * uu * imRV;
        acc[3] += 2.0 * ww * two_pi * vv * imRV;
        acc[4] += -2.0 * ww * (Rr * Ir2 + Ri * Ii2);
    }
    if (bad) atomicOr(&ctl->flag, STATUS_UV);
#pragma unroll
    for (int q = 0; q < GEO_N; ++q) {
        const double bs = block_sum(acc[q], red);
        if (threadIdx.x == 0) partials[(size_t)q * gridDim.x + blk] = bs;
    }
}

// the five sums, each over its row of partials in a fixed order (one block each)
__global__ __launch_bounds__(REDUCE_NT) void k_reduce_geo(const double *__restrict__ partials,
                                                          int nblk, double *__restrict__ chi2,
                                                          double *__restrict__ dgeo) {
    __shared__ double red[REDUCE_NT / 64];
    const int q = blockIdx.x;
    const double tot = block_sum(strided_sum(partials + (size_t)q * nblk, nblk), red);
    if (threadIdx.x == 0) {
        if (q == 0) *chi2 = tot;
        else dgeo[q - 1] = tot;
    }
}

}  // namespace gal
