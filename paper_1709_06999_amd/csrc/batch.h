// batch.h -- many chi^2 evaluations in one set of launches.
//
// A batch is a fixed list of jobs (model + dataset + image size).  Its
// structure is planned once on the host (gal_batch_create): jobs with the same
// precision, kind and image size share the FFT launches (one block row per
// job, blockIdx.y), and jobs on the same dataset share the sampling launch: a
// block loads its chunk of observations once and evaluates every job of its
// group on it, so the uv data is read once per group instead of once per job.
// Jobs of one scene are the sources of one field (Sec. 3.2: the visibilities
// of several sources add up): the sampling pass sums their visibilities at
// each point before the residual, and a source may read the spectrum of an
// identical source instead of transforming its own, so that copies of one
// model at other offsets and orientations cost one gather each and no FFT.
// The per-job geometry (Rmin, dR, inc, PA, dRA, dDec) and the model arrays
// are read from device memory at execution, so one plan (and a HIP graph
// captured from it) serves every step of a fitter that updates those buffers
// in place.
#pragma once
#include <type_traits>

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
    void *vis;           // visibilities of the job's scene [M] (c2, dataset precision), or NULL
    int kind;            // 0 image, 1 profile
    int N, Nr, Q, P, CS, Qe;
    double dxy;
    // constants of the job's geometry, written by kb_prepare at the head of
    // every execution (geo may change between executions)
    double cpa, spa, cinc, dRA, dDec;  // sampling
    double cpa_du, spa_du;             // cos PA, sin PA times N dxy
    double Rmin, inv_dR, inv_cos;      // sweep (profiles)
    int bad;                           // the geometry row failed its checks
    int shared;                        // reads another job's spectrum (share > 0)
};

// one thread per job: the trigonometry and divisions every later block of
// the job would otherwise repeat, and the checks the single calls make on the
// host (finite PA, inc, offsets, cos(inc) > 0; for profiles finite dR > 0 and
// Rmin >= 0).  A job that fails them is marked: its chi^2 (that of its scene)
// and its gradient come out NaN, and the status flag gets STATUS_GEO.
__global__ __launch_bounds__(64) void kb_prepare(JobDesc *__restrict__ jobs, int n,
                                                 Control *ctl) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    JobDesc &j = jobs[i];
    const double *geo = j.geo;
    double sn, cs;
    sincos(geo[3], &sn, &cs);
    const double ci = cos(geo[2]);
    // (a profile that reads another job's spectrum takes Rmin, dR and inc
    // from that job: its own are not used)
    const bool own_sweep = j.kind == 1 && !j.shared;
    bool ok = isfinite(geo[3]) && isfinite(geo[4]) && isfinite(geo[5]);
    if (j.kind == 0 || own_sweep) ok = ok && isfinite(geo[2]) && ci > 0.0;
    if (own_sweep) ok = ok && isfinite(geo[0]) && geo[0] >= 0.0 && isfinite(geo[1]) && geo[1] > 0.0;
    j.bad = ok ? 0 : 1;
    if (!ok) atomicOr(&ctl->flag, STATUS_GEO);
    j.cpa = cs;
    j.spa = sn;
    j.cpa_du = cs * ((double)j.N * j.dxy);
    j.spa_du = sn * ((double)j.N * j.dxy);
    j.cinc = j.kind == 1 ? 1.0 : ci;
    j.dRA = geo[4];
    j.dDec = geo[5];
    j.Rmin = geo[0];
    j.inv_dR = 1.0 / geo[1];
    j.inv_cos = 1.0 / ci;
}

struct SGroup {          // scenes sharing one pass over a dataset
    const void *u, *v, *re, *im, *w;  // re, im, w NULL: no observations (chi^2 = 0)
    const int32_t *perm;              // stored point -> registration index
    int64_t M;
    int blk0, nblk;      // flattened block range of the group
    int nchunk, cpb;     // chunks of SAMPLE_NT * SAMPLE_PPT points; chunks per block
    int job_off, nj;     // lists[job_off + m]: job indices, scene members adjacent
    int sc_off, nsc;     // lists[sc_off + s]: first member of scene s; [sc_off + nsc] = nj
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
    a.dxs = j.dxy * j.inv_cos;
    a.t0 = -j.Rmin * j.inv_dR;
    return a;
}

__device__ __forceinline__ SampleArgs sample_from_job(const JobDesc &j, int64_t M) {
    SampleArgs a;
    a.M = M;
    a.inv_du = (double)j.N * j.dxy;
    a.cpa = j.cpa;
    a.spa = j.spa;
    a.cinc = j.cinc;
    a.cpa_du = j.cpa_du;
    a.spa_du = j.spa_du;
    a.dRA = j.dRA;
    a.dDec = j.dDec;
    a.ph_u = 256.0 * j.dRA;
    a.ph_v = 256.0 * j.dDec;
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
__global__ __launch_bounds__(Cfg::NT) void kb_rows_even(const JobDesc *__restrict__ jobs,
                                                        const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    rows_even_body<T, Cfg, gptr<T>>(as_global<T>(j.src), sweep_of(j), geom_of(j), j.Qe,
                                    (T *)(ws + j.spec_off), xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_cols_sym(const JobDesc *__restrict__ jobs,
                                                       const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    cols_sym_body<T, Cfg>(geom_of(j), j.Qe, (T *)(ws + j.spec_off), blockIdx.x);
}

template <typename T, typename Cfg>
__global__ __launch_bounds__(Cfg::NT) void kb_cols_even(const JobDesc *__restrict__ jobs,
                                                        const int *__restrict__ list, char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    cols_even_body<T, Cfg>(geom_of(j), j.Qe, (T *)(ws + j.spec_off), blockIdx.x);
}

// ---- sampling stage ------------------------------------------------------
// One job at one point: the bilinear value of its spectrum (cos(inc) for
// images) times the phase of its offset, plus the stencil for a scatter.
template <typename T, bool REAL>
struct JobPoint {
    std::conditional_t<REAL, StencilE<T>, Stencil<T>> st;
    double Vre, Vim, sn, cs;
};

template <typename T, bool REAL>
__device__ __forceinline__ JobPoint<T, REAL> job_point(const JobDesc &J, const SampleArgs &a,
                                                       const Geom &g, const char *ws, double u,
                                                       double v) {
    JobPoint<T, REAL> r;
    // exp(i theta), theta = 2 pi (u dRA + v dDec)
    phase_of(a, u, v, r.sn, r.cs);
    // an off-grid stencil points at valid nodes; its value is discarded
    if constexpr (REAL) {
        r.st = locate_e<T>(g, a, u, v);
        const StencilE<T> &st = r.st;
        double x0, x1, y0, y1;
        nodes_e<T>((const T *)(ws + J.spec_off), st, g.CS, x0, x1, y0, y1);
        double b = bilerp(x0, y0, x1, y1, st.s, st.t);  // cos(inc) = 1 on real spectra
        b = st.ok ? b : __builtin_nan("");
        r.Vre = b * r.cs;
        r.Vim = b * r.sn;
    } else {
        r.st = locate<T>((const c2<T> *)(ws + J.spec_off), g, a, u, v);
        const Stencil<T> &st = r.st;
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
        r.Vre = st.ok ? br * r.cs - bi * r.sn : __builtin_nan("");
        r.Vim = st.ok ? br * r.sn + bi * r.cs : __builtin_nan("");
    }
    return r;
}

// the point's share of d chi^2 / d spectrum for residual R = obs - V (weight w)
template <typename T, bool REAL>
__device__ __forceinline__ PointAdd<REAL ? 1 : 2> job_point_add(const JobPoint<T, REAL> &q,
                                                                 double w, double cinc, double R0,
                                                                 double R1) {
    if constexpr (REAL) return point_add_real<T>(q.st, w * (R0 * q.cs + R1 * q.sn));  // cinc = 1
    else return point_add_cplx<T>(q.st, w * cinc, R0, R1, q.sn, q.cs);
}

template <typename T>
__device__ __forceinline__ void store_vis(void *vis, const int32_t *perm, int64_t k, double re,
                                          double im) {
    ((c2<T> *)vis)[perm ? (int64_t)perm[k] : k] = c2<T>{(T)re, (T)im};
}

// Points held by one thread of a sampling block.
template <int PPT, int64_t STEP>
struct BlockPoints {
    int64_t base, M;  // point p of the thread: base + p STEP
    double uu[PPT], vv[PPT], rr[PPT], ii[PPT], ww[PPT];
    __device__ __forceinline__ bool in(int p) const { return base + p * STEP < M; }
    __device__ __forceinline__ int64_t idx(int p) const { return base + p * STEP; }
};

// A job alone in its scene (of the scene kernel): value, residual, chi^2 term,
// visibility output and scatter in one sweep over the thread's points.
// Returns the thread's chi^2 sum.
template <typename T, bool REAL, bool GRAD, int PPT, int64_t STEP>
__device__ __forceinline__ double job_alone(const JobDesc &J, const BlockPoints<PPT, STEP> &X,
                                            const int32_t *perm, char *ws, double *tile,
                                            int *box, bool &bad) {
    constexpr int NV = REAL ? 1 : 2;
    const SampleArgs a = sample_from_job(J, X.M);
    const Geom g = geom_of(J);
    double acc = 0.0;
    PointAdd<NV> pa[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const bool in = X.in(p);
        pa[p].q = -1;
        const JobPoint<T, REAL> q = job_point<T, REAL>(J, a, g, ws, X.uu[p], X.vv[p]);
        if (GRAD && J.grad && in && q.st.ok)
            pa[p] = job_point_add<T, REAL>(q, X.ww[p], a.cinc, X.rr[p] - q.Vre, X.ii[p] - q.Vim);
        bad |= in && !q.st.ok;
        // (w = 0 past M, where the stencil at u = v = 0 is valid)
        const double dr = q.Vre - X.rr[p], di = q.Vim - X.ii[p];
        acc += X.ww[p] * (dr * dr + di * di);
        if (in && J.vis) store_vis<T>(J.vis, perm, X.idx(p), q.Vre, q.Vim);
    }
    if (GRAD && J.grad) block_scatter<T, NV, PPT>((T *)(ws + J.a_off), g.CS, pa, tile, box);
    return acc;
}

// V += the job's visibilities at the thread's points
template <typename T, bool REAL, int PPT, int64_t STEP>
__device__ __forceinline__ void job_add(const JobDesc &J, const BlockPoints<PPT, STEP> &X,
                                        const char *ws, double (&Vr)[PPT], double (&Vi)[PPT],
                                        bool &bad) {
    const SampleArgs a = sample_from_job(J, X.M);
    const Geom g = geom_of(J);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const JobPoint<T, REAL> q = job_point<T, REAL>(J, a, g, ws, X.uu[p], X.vv[p]);
        bad |= X.in(p) && !q.st.ok;
        Vr[p] += q.Vre;
        Vi[p] += q.Vim;
    }
}

// the job's part of d chi^2 / d spectrum for the scene's residual R
template <typename T, bool REAL, int PPT, int64_t STEP>
__device__ __forceinline__ void job_scatter(const JobDesc &J, const BlockPoints<PPT, STEP> &X,
                                            char *ws, const double (&Rr)[PPT],
                                            const double (&Ri)[PPT], double *tile, int *box) {
    constexpr int NV = REAL ? 1 : 2;
    const SampleArgs a = sample_from_job(J, X.M);
    const Geom g = geom_of(J);
    PointAdd<NV> pa[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        pa[p].q = -1;
        const JobPoint<T, REAL> q = job_point<T, REAL>(J, a, g, ws, X.uu[p], X.vv[p]);
        if (X.in(p) && q.st.ok) pa[p] = job_point_add<T, REAL>(q, X.ww[p], a.cinc, Rr[p], Ri[p]);
    }
    block_scatter<T, NV, PPT>((T *)(ws + J.a_off), g.CS, pa, tile, box);
}

// Plain groups (every job alone in its scene, with observations and no
// visibility output).  Block -> group by binary search over the groups' first
// blocks (after the XCD remap); each thread keeps SAMPLE_PPT points in
// registers and evaluates every job of the group.  GRAD: jobs with a gradient
// output also scatter their residuals.  MULTI: a block takes cpb consecutive
// chunks of its group (groups of few jobs, where one chunk is too little
// work to cover the block's set-up and memory latency), loading the next
// chunk's observations while it evaluates the current one.
template <typename T, bool REAL, bool GRAD, bool MULTI = false>
__global__ __launch_bounds__(SAMPLE_NT) void kb_sample_chi2(const JobDesc *__restrict__ jobs,
                                                            const SGroup *__restrict__ groups,
                                                            const int *__restrict__ lists,
                                                            int ngroups, char *ws) {
    static_assert(!(GRAD && MULTI), "one chunk per block with gradients");
    constexpr int PPT = SAMPLE_PPT;
    constexpr int NV = REAL ? 1 : 2;
    __shared__ double tile[GRAD ? SCAT_TILE : 1];
    __shared__ int box[GRAD ? 4 * WAVES : 1];
    // every XCD takes a contiguous run of chunks: a compact patch of the
    // (locality-ordered) uv plane, whose spectrum nodes then stay in its L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].blk0 <= bid) lo = mid;
        else hi = mid - 1;
    }
    const SGroup &G = groups[lo];
    const int c0 = MULTI ? (bid - G.blk0) * G.cpb : bid - G.blk0;
    const int c1 = MULTI ? min(c0 + G.cpb, G.nchunk) : c0 + 1;
    // chi^2 only: points strided by the block size (each load instruction
    // reads one contiguous run); with gradients: SAMPLE_PPT consecutive
    // points per thread, neighbours in the locality order of datasets, whose
    // equal stencils block_scatter folds in registers before the LDS atomics
    constexpr int64_t PSTEP = GRAD ? 1 : SAMPLE_NT;
    const gptr<T> u = as_global<T>(G.u), v = as_global<T>(G.v);
    const gptr<T> re = as_global<T>(G.re), im = as_global<T>(G.im), w = as_global<T>(G.w);
    auto first = [&](int chunk) {
        return (int64_t)chunk * (SAMPLE_NT * PPT) + threadIdx.x * (GRAD ? PPT : 1);
    };
    // the observations of a chunk as stored (points past M: 0, weight 0)
    T su[PPT], sv[PPT], sr[PPT], si[PPT], sw[PPT];
    auto fetch = [&](int chunk) {
        const int64_t b = first(chunk);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int64_t k = b + p * PSTEP;
            const bool in = k < G.M;
            su[p] = in ? u[k] : T(0);
            sv[p] = in ? v[k] : T(0);
            sr[p] = in ? re[k] : T(0);
            si[p] = in ? im[k] : T(0);
            sw[p] = in ? w[k] : T(0);  // points past M weigh nothing
        }
    };
    fetch(c0);
    Control *ctl = (Control *)ws;
    bool bad = false;
    for (int chunk = c0; chunk < c1; ++chunk) {
        const int64_t base = first(chunk);
        double uu[PPT], vv[PPT], rr[PPT], ii[PPT], ww[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            uu[p] = (double)su[p];
            vv[p] = (double)sv[p];
            rr[p] = (double)sr[p];
            ii[p] = (double)si[p];
            ww[p] = (double)sw[p];
        }
        if (MULTI && chunk + 1 < c1) fetch(chunk + 1);  // in flight during this chunk's jobs
        for (int jj = 0; jj < G.nj; ++jj) {
            const JobDesc &J = jobs[lists[G.job_off + jj]];
            const SampleArgs a = sample_from_job(J, G.M);
            const Geom g = geom_of(J);
            double acc = 0.0;
            PointAdd<NV> pa[PPT];
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const bool in = base + p * PSTEP < G.M;
                pa[p].q = -1;
                // exp(i theta), theta = 2 pi (u dRA + v dDec)
                double sn, cs;
                phase_of(a, uu[p], vv[p], sn, cs);
                double Vre, Vim;
                bool ok;
                // an off-grid stencil points at valid nodes; its value is discarded
                if constexpr (REAL) {
                    const T *S = (const T *)(ws + J.spec_off);
                    const StencilE<T> st = locate_e<T>(g, a, uu[p], vv[p]);
                    ok = st.ok;
                    double x0, x1, y0, y1;
                    nodes_e<T>(S, st, g.CS, x0, x1, y0, y1);
                    double b = bilerp(x0, y0, x1, y1, st.s, st.t);  // cos(inc) = 1 on real spectra
                    b = ok ? b : __builtin_nan("");
                    Vre = b * cs;
                    Vim = b * sn;
                    if (GRAD && J.grad && in && ok) {
                        // Re(conj(R) e^{i theta}) on the real spectrum
                        const double R0 = rr[p] - Vre, R1 = ii[p] - Vim;
                        pa[p] = point_add_real<T>(st, ww[p] * (R0 * cs + R1 * sn));
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
                // no branch on `in`: a point past M has w = 0 and a valid stencil
                // at u = v = 0 (finite V), so it adds 0, and the four points'
                // gathers can be in flight together
                const double dr = Vre - rr[p], di = Vim - ii[p];
                acc += ww[p] * (dr * dr + di * di);
            }
            if (GRAD && J.grad) block_scatter<T, NV, PPT>((T *)(ws + J.a_off), g.CS, pa, tile, box);
            // one partial per wave (no barrier between chi^2-only jobs); kb_reduce adds them
            const double wsum = wave_sum_permute(acc);
            if ((threadIdx.x & 63) == 0)
                ((double *)(ws + J.part_off))[chunk * WAVES + (threadIdx.x >> 6)] = wsum;
        }
    }
    if (bad) atomicOr(&ctl->flag, STATUS_UV);
}

// KC: the kinds of the class's jobs -- 0 images, 1 profiles, 2 both (the kind
// is then read per job; a uniform branch).
template <int KC>
__device__ __forceinline__ bool real_job(const JobDesc &J) {
    if constexpr (KC == 2) return J.kind == 1;
    else return KC == 1;
}

// Groups of scenes: several sources, visibility outputs or datasets without
// observations (a kernel of its own, so that the registers these need do not
// lower the occupancy of the plain one).  As kb_sample_chi2, per scene: the
// members' visibilities add up before the residual, and members with a
// gradient scatter the scene's residual.
template <typename T, int KC, bool GRAD>
__global__ __launch_bounds__(SAMPLE_NT) void kb_sample_scene(const JobDesc *__restrict__ jobs,
                                                            const SGroup *__restrict__ groups,
                                                            const int *__restrict__ lists,
                                                            int ngroups, char *ws) {
    constexpr int PPT = SAMPLE_PPT;
    __shared__ double tile[GRAD ? SCAT_TILE : 1];
    __shared__ int box[GRAD ? 4 * WAVES : 1];
    // every XCD takes a contiguous run of chunks: a compact patch of the
    // (locality-ordered) uv plane, whose spectrum nodes then stay in its L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].blk0 <= bid) lo = mid;
        else hi = mid - 1;
    }
    const SGroup &G = groups[lo];
    const int chunk = bid - G.blk0;
    // points strided by the block size, or consecutive with gradients (as
    // kb_sample_chi2)
    constexpr int64_t STEP = GRAD ? 1 : SAMPLE_NT;
    BlockPoints<PPT, STEP> X;
    X.base = (int64_t)chunk * (SAMPLE_NT * PPT) + threadIdx.x * (GRAD ? PPT : 1);
    X.M = G.M;
    const gptr<T> u = as_global<T>(G.u), v = as_global<T>(G.v);
    const gptr<T> re = as_global<T>(G.re), im = as_global<T>(G.im), w = as_global<T>(G.w);
    const bool obs = G.re != nullptr;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = X.idx(p);
        const bool in = k < G.M;
        X.uu[p] = in ? (double)u[k] : 0.0;
        X.vv[p] = in ? (double)v[k] : 0.0;
        X.rr[p] = in && obs ? (double)re[k] : 0.0;
        X.ii[p] = in && obs ? (double)im[k] : 0.0;
        X.ww[p] = in && obs ? (double)w[k] : 0.0;  // points past M weigh nothing
    }
    Control *ctl = (Control *)ws;
    bool bad = false;
    const int *mem = lists + G.job_off;
    for (int sc = 0; sc < G.nsc; ++sc) {
        const int m0 = lists[G.sc_off + sc], m1 = lists[G.sc_off + sc + 1];
        const JobDesc &L = jobs[mem[m0]];
        double acc = 0.0;
        if (m1 - m0 == 1) {
            if (real_job<KC>(L)) {
                if constexpr (KC != 0)
                    acc = job_alone<T, true, GRAD, PPT, STEP>(L, X, G.perm, ws, tile, box, bad);
            } else {
                if constexpr (KC != 1)
                    acc = job_alone<T, false, GRAD, PPT, STEP>(L, X, G.perm, ws, tile, box, bad);
            }
        } else {
            // a scene of several sources: V = sum of the sources' visibilities
            double Vr[PPT], Vi[PPT];
#pragma unroll
            for (int p = 0; p < PPT; ++p) Vr[p] = Vi[p] = 0.0;
            for (int m = m0; m < m1; ++m) {
                const JobDesc &J = jobs[mem[m]];
                if (real_job<KC>(J)) {
                    if constexpr (KC != 0) job_add<T, true, PPT, STEP>(J, X, ws, Vr, Vi, bad);
                } else {
                    if constexpr (KC != 1) job_add<T, false, PPT, STEP>(J, X, ws, Vr, Vi, bad);
                }
            }
#pragma unroll
            for (int p = 0; p < PPT; ++p) {  // w = 0 past M
                const double dr = Vr[p] - X.rr[p], di = Vi[p] - X.ii[p];
                acc += X.ww[p] * (dr * dr + di * di);
            }
            for (int m = m0; m < m1; ++m) {
                const JobDesc &J = jobs[mem[m]];
                if (!J.vis) continue;
#pragma unroll
                for (int p = 0; p < PPT; ++p)
                    if (X.in(p)) store_vis<T>(J.vis, G.perm, X.idx(p), Vr[p], Vi[p]);
            }
            if constexpr (GRAD) {
                double Rr[PPT], Ri[PPT];
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    Rr[p] = X.rr[p] - Vr[p];
                    Ri[p] = X.ii[p] - Vi[p];
                }
                for (int m = m0; m < m1; ++m) {
                    const JobDesc &J = jobs[mem[m]];
                    if (!J.grad) continue;
                    if (real_job<KC>(J)) {
                        if constexpr (KC != 0) job_scatter<T, true, PPT, STEP>(J, X, ws, Rr, Ri, tile, box);
                    } else {
                        if constexpr (KC != 1) job_scatter<T, false, PPT, STEP>(J, X, ws, Rr, Ri, tile, box);
                    }
                }
            }
        }
        // one partial per wave and scene (no barrier between chi^2-only
        // scenes); kb_reduce adds them
        const double wsum = wave_sum_permute(acc);
        if ((threadIdx.x & 63) == 0)
            ((double *)(ws + L.part_off))[chunk * WAVES + (threadIdx.x >> 6)] = wsum;
    }
    if (bad) atomicOr(&ctl->flag, STATUS_UV);
}

// chi2[j] = sum of the partials of job j's scene in a fixed order (one block
// per job, as k_reduce).  Bitwise repeatable.  NaN when a job of the scene
// (the jobs sharing its partials) failed the geometry checks of kb_prepare.
__global__ __launch_bounds__(REDUCE_NT) void kb_reduce(const JobDesc *__restrict__ jobs, int njobs,
                                                       const SGroup *__restrict__ groups,
                                                       const int *__restrict__ job_group,
                                                       const char *ws, double *__restrict__ chi2) {
    __shared__ double red[REDUCE_NT / 64];
    __shared__ int any_bad;
    const int j = blockIdx.x;
    const JobDesc &J = jobs[j];
    if (threadIdx.x == 0) any_bad = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < njobs; k += REDUCE_NT)
        if (jobs[k].bad && jobs[k].part_off == J.part_off) any_bad = 1;
    const int n = groups[job_group[j]].nchunk * WAVES;
    const double tot = block_sum(strided_sum((const double *)(ws + J.part_off), n), red);
    if (threadIdx.x == 0) chi2[j] = any_bad ? __builtin_nan("") : tot;
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
    adj_rows_body<T, Cfg>(geom_of(j), (const c2<T> *)(ws + j.a_off), (T *)j.grad,
                          xcd_remap(blockIdx.x, gridDim.x), j.bad != 0);
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
                                                           char *ws, int ppb) {
    extern __shared__ double hist[];
    const JobDesc &j = jobs[list[blockIdx.y]];
    adj_rows_sym_body<T, Cfg>(geom_of(j), (const T *)(ws + j.a_off), sweep_of(j),
                              (double *)(ws + j.gi_off) + (size_t)(blockIdx.x % GI_COPIES) * j.Nr,
                              hist, xcd_remap(blockIdx.x, gridDim.x), ppb);
}

// profile gradients: the sum of the accumulator copies into the caller's array
template <typename T>
__global__ __launch_bounds__(256) void kb_grad_out(const JobDesc *__restrict__ jobs,
                                                   const int *__restrict__ list, const char *ws) {
    const JobDesc &j = jobs[list[blockIdx.y]];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < j.Nr) {
        sum_bins<T>((const double *)(ws + j.gi_off), j.Nr, (T *)j.grad, i);
        if (j.bad) ((T *)j.grad)[i] = T(__builtin_nan(""));
    }
}

}  // namespace gal
