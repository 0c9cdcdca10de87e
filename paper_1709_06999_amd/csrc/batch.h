// batch.h -- many chi^2 evaluations in one set of launches.
//
// A batch is a fixed list of jobs (model + dataset + image size).  Its
// structure is planned once on the host (gal_batch_create): jobs with the same
// precision, kind and image size share the FFT launches (one block row per
// job, blockIdx.y), and jobs on the same dataset, kind and image grid share
// the sampling launch: a block loads its chunk of observations once and
// evaluates every job of its group on it, so the uv data is read once per
// group instead of once per job.  The per-job geometry (Rmin, dR, inc, PA,
// dRA, dDec) and the model arrays are read from device memory at execution,
// so one plan (and a HIP graph captured from it) serves every step of a
// fitter that updates those buffers in place.
#pragma once
#include "adjoint.h"
#include "kernels.h"

namespace gal {

constexpr int KMAX = 16;  // jobs sharing one pass over a dataset
constexpr int WAVES = SAMPLE_NT / 64;  // chi^2 partials per sampling block and job

struct JobDesc {
    const void *src;     // image [N*N] or profile [Nr], dataset precision
    const double *geo;   // Rmin, dR, inc, PA, dRA, dDec
    void *grad;          // gradient output (dataset precision), NULL: chi^2 only
    size_t spec_off;     // spectrum slot: byte offset in the workspace
    size_t part_off;     // partial sums: byte offset in the workspace
    size_t a_off;        // scatter grid of a gradient job
    size_t gi_off;       // profile-bin accumulator (double) of a gradient profile job
    int kind;            // 0 image, 1 profile
    int N, Nr, Q, P, CS, Qe;
    double dxy;
    // constants of the job's geometry, written by kb_prepare at the head of
    // every execution (geo may change between executions)
    double cpa, spa, cinc, dRA, dDec;  // sampling
    double Rmin, inv_dR, inv_cos;      // sweep (profiles)
};

// one thread per job: the trigonometry and divisions every later block of
// the job would otherwise repeat
__global__ __launch_bounds__(64) void kb_prepare(JobDesc *__restrict__ jobs, int n) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    JobDesc &j = jobs[i];
    const double *geo = j.geo;
    double sn, cs;
    sincos(geo[3], &sn, &cs);
    const double ci = cos(geo[2]);
    j.cpa = cs;
    j.spa = sn;
    j.cinc = j.kind == 1 ? 1.0 : ci;
    j.dRA = geo[4];
    j.dDec = geo[5];
    j.Rmin = geo[0];
    j.inv_dR = 1.0 / geo[1];
    j.inv_cos = 1.0 / ci;
}

struct SGroup {          // jobs sharing one pass over a dataset
    const void *u, *v, *re, *im, *w;
    int64_t M;
    int blk0, nblk;      // flattened block range of the group
    int nj;
    int jobs[KMAX];
};

__device__ __forceinline__ SweepArgs sweep_of(const JobDesc &j) {
    SweepArgs a;
    a.Nr = j.Nr;
    a.Rmin = j.Rmin;
    a.inv_dR = j.inv_dR;
    a.dxy = j.dxy;
    a.inv_cos = j.inv_cos;
    a.pix_area = j.dxy * j.dxy;
    a.tmax = (double)(j.Nr - 1);
    return a;
}

__device__ __forceinline__ SampleArgs sample_from_job(const JobDesc &j, int64_t M) {
    SampleArgs a;
    a.M = M;
    a.inv_du = (double)j.N * j.dxy;
    a.cpa = j.cpa;
    a.spa = j.spa;
    a.cinc = j.cinc;
    a.dRA = j.dRA;
    a.dDec = j.dDec;
    a.jmax = min(j.Q - 2, j.N / 2 - 1);
    a.imin = -min(j.P, j.N / 2);
    a.imax = min(j.P - 1, j.N / 2 - 2);
    return a;
}

__device__ __forceinline__ Geom geom_of(const JobDesc &j) { return Geom{j.N, j.Q, j.P, j.CS}; }

// ---- FFT stage: blockIdx.y selects the job in `list` ----------------------
template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_rows_img(const JobDesc *__restrict__ jobs,
                                                       const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    rows_body<T, Cfg, false>((const T *)j.src, SweepArgs{}, geom_of(j),
                             (c2<T> *)(ws + j.spec_off), xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_cols(const JobDesc *__restrict__ jobs,
                                                   const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    cols_body<T, Cfg>(geom_of(j), (c2<T> *)(ws + j.spec_off), blockIdx.x);
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_rows_sym(const JobDesc *__restrict__ jobs,
                                                       const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    rows_sym_body<T, Cfg, gptr<T>>(as_global<T>(j.src), sweep_of(j), geom_of(j), j.Qe,
                                   (T *)(ws + j.spec_off), xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_cols_sym(const JobDesc *__restrict__ jobs,
                                                       const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    cols_sym_body<T, Cfg>(geom_of(j), j.Qe, (T *)(ws + j.spec_off), blockIdx.x);
}

// ---- sampling stage ------------------------------------------------------
// Block -> group by binary search over the groups' first blocks (after the
// XCD remap); each thread
// keeps SAMPLE_PPT points in registers and evaluates every job of the group.
// GRAD: jobs with a gradient output also scatter their residuals.
template <typename T, bool REAL, bool GRAD>
__global__ __launch_bounds__(SAMPLE_NT) void kb_sample_chi2(const JobDesc *__restrict__ jobs,
                                                            const SGroup *__restrict__ groups,
                                                            int ngroups, char *ws) {
    constexpr int PPT = SAMPLE_PPT;
    constexpr int NV = REAL ? 1 : 2;
    __shared__ double tile[GRAD ? SCAT_TILE : 1];
    __shared__ int box[GRAD ? 4 * WAVES : 1];
    // every XCD takes a contiguous run of chunks: a compact patch of the
    // (Morton-ordered) uv plane, whose spectrum nodes then stay in its L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].blk0 <= bid) lo = mid;
        else hi = mid - 1;
    }
    const SGroup &G = groups[lo];
    const int chunk = bid - G.blk0;
    const int64_t base = (int64_t)chunk * (SAMPLE_NT * PPT) + threadIdx.x;
    const gptr<T> u = as_global<T>(G.u), v = as_global<T>(G.v);
    const gptr<T> re = as_global<T>(G.re), im = as_global<T>(G.im), w = as_global<T>(G.w);
    double uu[PPT], vv[PPT], rr[PPT], ii[PPT], ww[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = base + p * SAMPLE_NT;
        const bool in = k < G.M;
        uu[p] = in ? (double)u[k] : 0.0;
        vv[p] = in ? (double)v[k] : 0.0;
        rr[p] = in ? (double)re[k] : 0.0;
        ii[p] = in ? (double)im[k] : 0.0;
        ww[p] = in ? (double)w[k] : 0.0;  // points past M weigh nothing
    }
    Control *ctl = (Control *)ws;
    bool bad = false;
    for (int jj = 0; jj < G.nj; ++jj) {
        const JobDesc &J = jobs[G.jobs[jj]];
        const SampleArgs a = sample_from_job(J, G.M);
        const Geom g = geom_of(J);
        double acc = 0.0;
        PointAdd<NV> pa[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const bool in = base + p * SAMPLE_NT < G.M;
            pa[p].q = -1;
            // exp(i theta), theta = 2 pi (u dRA + v dDec)
            double sn, cs;
            sincospi_tab(2.0 * (uu[p] * a.dRA + vv[p] * a.dDec), sn, cs);
            double Vre, Vim;
            bool ok;
            // an off-grid stencil points at valid nodes; its value is discarded
            if constexpr (REAL) {
                const T *S = (const T *)(ws + J.spec_off);
                const StencilR<T> st = locate_r<T>(S, g, a, uu[p], vv[p]);
                ok = st.ok;
                const T x0 = st.c0[0], x1 = st.c0[1], y0 = st.c0[g.CS], y1 = st.c0[g.CS + 1];
                const double a00 = st.swap ? x1 : x0, a10 = st.swap ? x0 : x1;
                const double a01 = st.swap ? y1 : y0, a11 = st.swap ? y0 : y1;
                const double s = st.s, t = st.t;
                const double b = a.cinc * ((1.0 - t) * ((1.0 - s) * a00 + s * a01) +
                                           t * ((1.0 - s) * a10 + s * a11));
                Vre = ok ? b * cs : __builtin_nan("");
                Vim = ok ? b * sn : __builtin_nan("");
                if (GRAD && J.grad && in && ok) {
                    // Re(conj(R) e^{i theta}) on the real spectrum
                    const double R0 = rr[p] - Vre, R1 = ii[p] - Vim;
                    pa[p] = point_add_real<T>(st, ww[p] * a.cinc * (R0 * cs + R1 * sn));
                }
            } else {
                const c2<T> *S = (const c2<T> *)(ws + J.spec_off);
                const Stencil<T> st = locate<T>(S, g, a, uu[p], vv[p]);
                ok = st.ok;
                const c2<T> n00 = st.c0[0], n10 = st.c0[1], n01 = st.c0[g.CS], n11 = st.c0[g.CS + 1];
                const double s = st.s, t = st.t;
                const double w00 = (1.0 - t) * (1.0 - s), w01 = (1.0 - t) * s;
                const double w10 = t * (1.0 - s), w11 = t * s;
                double br = w00 * (double)n00.x + w01 * (double)n01.x + w10 * (double)n10.x +
                            w11 * (double)n11.x;
                double bi = w00 * (double)n00.y + w01 * (double)n01.y + w10 * (double)n10.y +
                            w11 * (double)n11.y;
                if (st.mirror) bi = -bi;
                br *= a.cinc;
                bi *= a.cinc;
                Vre = ok ? br * cs - bi * sn : __builtin_nan("");
                Vim = ok ? br * sn + bi * cs : __builtin_nan("");
                if (GRAD && J.grad && in && ok)
                    pa[p] = point_add_cplx<T>(st, ww[p] * a.cinc, rr[p] - Vre, ii[p] - Vim, sn, cs);
            }
            bad |= in && !ok;
            if (in) {
                const double dr = Vre - rr[p], di = Vim - ii[p];
                acc += ww[p] * (dr * dr + di * di);
            }
        }
        if (GRAD && J.grad) block_scatter<T, NV, PPT>((T *)(ws + J.a_off), g.CS, pa, tile, box);
        // one partial per wave (no barrier between chi^2-only jobs); kb_reduce adds them
        const double wsum = wave_sum(acc);
        if ((threadIdx.x & 63) == 0)
            ((double *)(ws + J.part_off))[chunk * WAVES + (threadIdx.x >> 6)] = wsum;
    }
    if (bad) ctl->flag = 1;
}

// chi2[j] = sum of job j's partials in a fixed order (one block per job,
// as k_reduce).  Bitwise repeatable.
__global__ __launch_bounds__(REDUCE_NT) void kb_reduce(const JobDesc *__restrict__ jobs,
                                                       const SGroup *__restrict__ groups,
                                                       const int *__restrict__ job_group,
                                                       const char *ws, double *__restrict__ chi2) {
    __shared__ double red[REDUCE_NT / 64];
    const int j = blockIdx.x;
    const JobDesc &J = jobs[j];
    const int n = groups[job_group[j]].nblk * WAVES;
    const double tot = block_sum(strided_sum((const double *)(ws + J.part_off), n), red);
    if (threadIdx.x == 0) chi2[j] = tot;
}

// ---- adjoint passes of gradient jobs: blockIdx.y selects the job ------------
template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_adj_cols(const JobDesc *__restrict__ jobs,
                                                       const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    adj_cols_body<T, Cfg>(geom_of(j), (c2<T> *)(ws + j.a_off), blockIdx.x);
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_adj_rows(const JobDesc *__restrict__ jobs,
                                                       const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    adj_rows_body<T, Cfg>(geom_of(j), (const c2<T> *)(ws + j.a_off), (T *)j.grad, blockIdx.x);
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_adj_cols_sym(const JobDesc *__restrict__ jobs,
                                                           const int *__restrict__ list,
                                                           char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    adj_cols_sym_body<T, Cfg>(geom_of(j), j.Qe, (T *)(ws + j.a_off), blockIdx.x);
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_adj_rows_sym(const JobDesc *__restrict__ jobs,
                                                           const int *__restrict__ list,
                                                           char *ws) {
    extern __shared__ double hist[];
    const JobDesc &j = jobs[list[blockIdx.y]];
    adj_rows_sym_body<T, Cfg>(geom_of(j), (const T *)(ws + j.a_off), sweep_of(j),
                              (double *)(ws + j.gi_off) + (size_t)(blockIdx.x % GI_COPIES) * j.Nr,
                              hist, blockIdx.x);
}

// profile gradients: the sum of the accumulator copies into the caller's array
template <typename T>
__global__ __launch_bounds__(256) void kb_grad_out(const JobDesc *__restrict__ jobs,
                                                   const int *__restrict__ list, const char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < j.Nr) sum_bins<T>((const double *)(ws + j.gi_off), j.Nr, (T *)j.grad, i);
}

}  // namespace gal
