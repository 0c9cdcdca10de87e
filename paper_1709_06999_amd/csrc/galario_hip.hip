// galario_hip.hip -- host side of the C ABI declared in include/galario_hip.h.
//
// Argument checks, the choice of which part of the half spectrum to
// transform, workspace carving, kernel launches and per-kernel timing.  All
// arithmetic of the path runs in the kernels of kernels.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <utility>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/galario_hip.h"
#include "kernels.h"

namespace gal {

__device__ c2<double> g_tw_d[2 * TW_MAX];
__device__ c2<float> g_tw_f[2 * TW_MAX];

// ---------------------------------------------------------------------------
// errors
static thread_local std::string t_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

#define GAL_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(GAL_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// twiddle tables: entries [M, 2M) hold exp(-2 pi i m / M) for every power of two M
static std::mutex g_init_mu;
static std::vector<char> g_init_done;

static int init_device(int dev) {
    std::lock_guard<std::mutex> lk(g_init_mu);
    if ((int)g_init_done.size() <= dev) g_init_done.resize(dev + 1, 0);
    if (g_init_done[dev]) return GAL_OK;
    std::vector<c2<double>> td(2 * TW_MAX);
    std::vector<c2<float>> tf(2 * TW_MAX);
    td[0] = {1.0, 0.0};
    tf[0] = {1.0f, 0.0f};
    const long double two_pi = 6.283185307179586476925286766559L;
    for (int M = 1; M <= TW_MAX; M *= 2) {
        for (int m = 0; m < M; ++m) {
            const long double a = two_pi * (long double)m / (long double)M;
            const double c = (double)cosl(a), s = (double)(-sinl(a));
            td[M + m] = {c, s};
            tf[M + m] = {(float)c, (float)s};
        }
    }
    int cur = 0;
    GAL_HIP(hipGetDevice(&cur));
    if (cur != dev) GAL_HIP(hipSetDevice(dev));
    GAL_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_tw_d), td.data(), sizeof(c2<double>) * td.size()));
    GAL_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_tw_f), tf.data(), sizeof(c2<float>) * tf.size()));
    if (cur != dev) GAL_HIP(hipSetDevice(cur));
    g_init_done[dev] = 1;
    return GAL_OK;
}

static int ensure_init() {
    int dev = 0;
    GAL_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_init_mu);
        if ((int)g_init_done.size() > dev && g_init_done[dev]) return GAL_OK;
    }
    return init_device(dev);
}

// ---------------------------------------------------------------------------
// per-kernel timing with HIP events on the launch stream
struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};
static std::mutex g_tm_mu;
static bool g_tm_on = false;
static std::vector<TimingRec> g_tm_recs;
static std::vector<hipEvent_t> g_tm_pool;

static hipEvent_t tm_event() {
    if (!g_tm_pool.empty()) {
        hipEvent_t e = g_tm_pool.back();
        g_tm_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct TimedLaunch {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    TimedLaunch(const char *n, hipStream_t st) : name(n), s(st) {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        if (!g_tm_on) return;
        a = tm_event();
        if (a) (void)hipEventRecord(a, s);
    }
    ~TimedLaunch() {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_tm_mu);
        hipEvent_t b = tm_event();
        if (!b) return;
        (void)hipEventRecord(b, s);
        g_tm_recs.push_back({name, a, b});
    }
};

static int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GAL_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return GAL_OK;
}

// ---------------------------------------------------------------------------
// per-size FFT shapes: rows (B rows of length N/2 per block, NT threads) and
// columns (B columns of length N per block, NT threads)
template <int N>
struct RowShape;
template <> struct RowShape<16> { static constexpr int B = 16, NT = 16; };
template <> struct RowShape<32> { static constexpr int B = 32, NT = 32; };
template <> struct RowShape<64> { static constexpr int B = 32, NT = 64; };
template <> struct RowShape<128> { static constexpr int B = 16, NT = 64; };
template <> struct RowShape<256> { static constexpr int B = 16, NT = 128; };
template <> struct RowShape<512> { static constexpr int B = 8, NT = 128; };
template <> struct RowShape<1024> { static constexpr int B = 4, NT = 128; };
template <> struct RowShape<2048> { static constexpr int B = 4, NT = 256; };
template <> struct RowShape<4096> { static constexpr int B = 2, NT = 256; };
template <> struct RowShape<8192> { static constexpr int B = 1, NT = 256; };

template <int N>
struct ColShape;
template <> struct ColShape<16> { static constexpr int B = 8, NT = 16; };
template <> struct ColShape<32> { static constexpr int B = 8, NT = 32; };
template <> struct ColShape<64> { static constexpr int B = 8, NT = 32; };
template <> struct ColShape<128> { static constexpr int B = 8, NT = 64; };
template <> struct ColShape<256> { static constexpr int B = 4, NT = 64; };
template <> struct ColShape<512> { static constexpr int B = 2, NT = 64; };
template <> struct ColShape<1024> { static constexpr int B = 1, NT = 64; };
template <> struct ColShape<2048> { static constexpr int B = 1, NT = 128; };
template <> struct ColShape<4096> { static constexpr int B = 1, NT = 256; };
template <> struct ColShape<8192> { static constexpr int B = 1, NT = 512; };

constexpr int min_c(int a, int b) { return a < b ? a : b; }

template <typename T, int L, int B, int NT>
using AutoCfg = FFTCfg<T, L, B, NT, min_c(16, min_c(B * L / NT, L))>;

template <typename T, int N>
using RowCfg = AutoCfg<T, N / 2, RowShape<N>::B, RowShape<N>::NT>;
template <typename T, int N>
using ColCfg = AutoCfg<T, N, ColShape<N>::B, ColShape<N>::NT>;

// Launch the two FFT passes for one image: src is the image (PROFILE false)
// or the profile (PROFILE true); result in XT with geometry g.
template <typename T, int N>
static int launch_fft(const T *src, bool profile, const SweepArgs &sw, const Geom &g, c2<T> *XT,
                      hipStream_t s) {
    using RC = RowCfg<T, N>;
    using CC = ColCfg<T, N>;
    {
        const dim3 grid(N / RC::B);
        if (profile) {
            TimedLaunch tl("k_rows_profile", s);
            k_rows<T, RC, true><<<grid, RC::NT, 0, s>>>(src, sw, g, XT);
        } else {
            TimedLaunch tl("k_rows_image", s);
            k_rows<T, RC, false><<<grid, RC::NT, 0, s>>>(src, sw, g, XT);
        }
        int rc = check_launch();
        if (rc) return rc;
    }
    {
        const dim3 grid((g.Q + CC::B - 1) / CC::B);
        TimedLaunch tl("k_cols", s);
        k_cols<T, CC><<<grid, CC::NT, 0, s>>>(g, XT);
    }
    return check_launch();
}

template <typename T>
static int dispatch_fft(int N, const T *src, bool profile, const SweepArgs &sw, const Geom &g,
                        c2<T> *XT, hipStream_t s) {
    switch (N) {
        case 16: return launch_fft<T, 16>(src, profile, sw, g, XT, s);
        case 32: return launch_fft<T, 32>(src, profile, sw, g, XT, s);
        case 64: return launch_fft<T, 64>(src, profile, sw, g, XT, s);
        case 128: return launch_fft<T, 128>(src, profile, sw, g, XT, s);
        case 256: return launch_fft<T, 256>(src, profile, sw, g, XT, s);
        case 512: return launch_fft<T, 512>(src, profile, sw, g, XT, s);
        case 1024: return launch_fft<T, 1024>(src, profile, sw, g, XT, s);
        case 2048: return launch_fft<T, 2048>(src, profile, sw, g, XT, s);
        case 4096: return launch_fft<T, 4096>(src, profile, sw, g, XT, s);
        case 8192: return launch_fft<T, 8192>(src, profile, sw, g, XT, s);
        default: return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", N);
    }
}

// Swept-profile transform (real, even spectrum): rows r in [0, N/2] in pairs,
// then column pairs; result SR[q * CS + p], p in [0, P], q in [0, Qe).
template <typename T, int N>
static int launch_fft_sym(const T *I, const SweepArgs &sw, const Geom &g, int Qe, T *XR,
                          hipStream_t s) {
    using CC = ColCfg<T, N>;
    {
        const int pairs = N / 4 + 1;
        const dim3 grid((pairs + CC::B - 1) / CC::B);
        TimedLaunch tl("k_rows_sym", s);
        k_rows_sym<T, CC><<<grid, CC::NT, 0, s>>>(I, sw, g, Qe, XR);
    }
    int rc = check_launch();
    if (rc) return rc;
    {
        const int pairs = Qe / 2;
        const dim3 grid((pairs + CC::B - 1) / CC::B);
        TimedLaunch tl("k_cols_sym", s);
        k_cols_sym<T, CC><<<grid, CC::NT, 0, s>>>(g, Qe, XR);
    }
    return check_launch();
}

template <typename T>
static int dispatch_fft_sym(int N, const T *I, const SweepArgs &sw, const Geom &g, int Qe, T *XR,
                            hipStream_t s) {
    switch (N) {
        case 16: return launch_fft_sym<T, 16>(I, sw, g, Qe, XR, s);
        case 32: return launch_fft_sym<T, 32>(I, sw, g, Qe, XR, s);
        case 64: return launch_fft_sym<T, 64>(I, sw, g, Qe, XR, s);
        case 128: return launch_fft_sym<T, 128>(I, sw, g, Qe, XR, s);
        case 256: return launch_fft_sym<T, 256>(I, sw, g, Qe, XR, s);
        case 512: return launch_fft_sym<T, 512>(I, sw, g, Qe, XR, s);
        case 1024: return launch_fft_sym<T, 1024>(I, sw, g, Qe, XR, s);
        case 2048: return launch_fft_sym<T, 2048>(I, sw, g, Qe, XR, s);
        case 4096: return launch_fft_sym<T, 4096>(I, sw, g, Qe, XR, s);
        case 8192: return launch_fft_sym<T, 8192>(I, sw, g, Qe, XR, s);
        default: return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", N);
    }
}

// ---------------------------------------------------------------------------
// workspace: [control 256 B][partials][XT]
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int64_t sample_blocks(int64_t M) {
    const int64_t per = (int64_t)SAMPLE_NT * SAMPLE_PPT;
    const int64_t n = (M + per - 1) / per;
    return n < 1 ? 1 : n;
}

template <typename T>
static size_t ws_bytes(int N, int64_t M) {
    const size_t partials = align256((size_t)sample_blocks(M) * sizeof(double));
    const size_t xt = align256((size_t)(N / 2 + 1) * (size_t)(N + 2) * sizeof(c2<T>));
    return 256 + partials + xt;
}

struct WS {
    Control *ctl;
    double *partials;
    void *xt;
};

template <typename T>
static int carve(void *ws, size_t bytes, int N, int64_t M, WS &out) {
    if (!ws) return fail(GAL_ERR_NULL, "workspace is NULL");
    const size_t need = ws_bytes<T>(N, M);
    if (bytes < need)
        return fail(GAL_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", bytes, need);
    char *p = (char *)ws;
    out.ctl = (Control *)p;
    out.partials = (double *)(p + 256);
    out.xt = p + 256 + align256((size_t)sample_blocks(M) * sizeof(double));
    return GAL_OK;
}

// ---------------------------------------------------------------------------
// argument checks
static bool pow2_in_range(int N) { return N >= 16 && N <= 8192 && (N & (N - 1)) == 0; }

static int check_image_scalars(int N, double dxy, double PA, double dRA, double dDec, double inc) {
    if (!pow2_in_range(N)) return fail(GAL_ERR_SIZE, "Nxy=%d: need a power of two in [16, 8192]", N);
    if (!(dxy > 0.0) || !std::isfinite(dxy)) return fail(GAL_ERR_SCALAR, "dxy must be > 0");
    if (!std::isfinite(PA) || !std::isfinite(dRA) || !std::isfinite(dDec) || !std::isfinite(inc))
        return fail(GAL_ERR_SCALAR, "PA, dRA, dDec and inc must be finite");
    if (!(std::cos(inc) > 0.0)) return fail(GAL_ERR_SCALAR, "cos(inc) must be > 0");
    return GAL_OK;
}

static int check_profile(int Nr, double Rmin, double dR) {
    if (Nr < 2) return fail(GAL_ERR_SIZE, "Nr=%d: need at least 2 radial samples", Nr);
    if (!(dR > 0.0) || !std::isfinite(dR)) return fail(GAL_ERR_SCALAR, "dR must be > 0");
    if (!(Rmin >= 0.0) || !std::isfinite(Rmin)) return fail(GAL_ERR_SCALAR, "Rmin must be >= 0");
    return GAL_OK;
}

static SweepArgs make_sweep(int Nr, double Rmin, double dR, double dxy, double inc) {
    SweepArgs a;
    a.Nr = Nr;
    a.Rmin = Rmin;
    a.inv_dR = 1.0 / dR;
    a.dxy = dxy;
    a.inv_cos = 1.0 / std::cos(inc);
    a.pix_area = dxy * dxy;
    a.tmax = (double)(Nr - 1);
    return a;
}

static Geom geom_full(int N) { return Geom{N, N / 2 + 1, N / 2, N + 2}; }

// the part of the spectrum that points with sqrt(u^2+v^2) <= rho_max reach
static Geom geom_pruned(int N, double dxy, double rho_max) {
    const double m = std::floor(rho_max * (double)N * dxy * (1.0 + 1e-12)) + 2.0;
    Geom g = geom_full(N);
    if (m < (double)g.Q) g.Q = (int)m;
    if (m < (double)g.P) g.P = (int)m;
    if (g.Q < 2) g.Q = 2;
    if (g.P < 1) g.P = 1;
    return g;
}

static SampleArgs make_sample(const Geom &g, int64_t M, double dxy, double PA, double dRA,
                              double dDec, double inc) {
    SampleArgs a;
    a.M = M;
    a.inv_du = (double)g.N * dxy;
    a.cpa = std::cos(PA);
    a.spa = std::sin(PA);
    a.cinc = std::cos(inc);
    a.dRA = dRA;
    a.dDec = dDec;
    a.jmax = min_c(g.Q - 2, g.N / 2 - 1);
    a.imin = -min_c(g.P, g.N / 2);
    a.imax = min_c(g.P - 1, g.N / 2 - 2);
    return a;
}

// ---------------------------------------------------------------------------
// the common path: (image | profile) -> spectrum -> samples -> (V | chi2)
template <typename T>
struct Obs {
    const T *u, *v, *re, *im, *w;
    int64_t M;
    const int32_t *perm;  // stored point k -> output slot perm[k] (NULL: k)
};

template <typename T>
static int run_path(const T *src, bool profile, const SweepArgs &sw, const Geom &g, double dxy,
                    const Obs<T> &o, double PA, double dRA, double dDec, double inc, T *vis,
                    double *chi2, void *ws, size_t ws_bytes_, hipStream_t s) {
    int rc = ensure_init();
    if (rc) return rc;
    WS w;
    rc = carve<T>(ws, ws_bytes_, g.N, o.M, w);
    if (rc) return rc;
    const SampleArgs sa = make_sample(g, o.M, dxy, PA, dRA, dDec, inc);
    const dim3 grid((unsigned)sample_blocks(o.M));
    if (profile) {
        // real spectrum of the (even) swept image, stored per column with stride N/2 + 2
        Geom gr = g;
        gr.CS = g.N / 2 + 2;
        const int Qe = (g.Q + 1) & ~1;
        T *XR = (T *)w.xt;
        rc = dispatch_fft_sym<T>(g.N, src, sw, gr, Qe, XR, s);
        if (rc) return rc;
        if (chi2) {
            {
                TimedLaunch tl("k_sample_sym_chi2", s);
                k_sample_sym<T, true><<<grid, SAMPLE_NT, 0, s>>>(XR, gr, sa, o.u, o.v, o.re, o.im,
                                                                 o.w, nullptr, nullptr, w.partials,
                                                                 w.ctl);
            }
            rc = check_launch();
            if (rc) return rc;
            TimedLaunch tl("k_reduce", s);
            k_reduce<<<1, SAMPLE_NT, 0, s>>>(w.partials, (int)grid.x, chi2);
        } else {
            TimedLaunch tl("k_sample_sym_vis", s);
            k_sample_sym<T, false><<<grid, SAMPLE_NT, 0, s>>>(XR, gr, sa, o.u, o.v, nullptr,
                                                              nullptr, nullptr, (c2<T> *)vis,
                                                              o.perm, w.partials, w.ctl);
        }
        return check_launch();
    }
    c2<T> *XT = (c2<T> *)w.xt;
    rc = dispatch_fft<T>(g.N, src, profile, sw, g, XT, s);
    if (rc) return rc;
    if (chi2) {
        {
            TimedLaunch tl("k_sample_chi2", s);
            k_sample<T, true><<<grid, SAMPLE_NT, 0, s>>>(XT, g, sa, o.u, o.v, o.re, o.im, o.w,
                                                         nullptr, nullptr, w.partials, w.ctl);
        }
        rc = check_launch();
        if (rc) return rc;
        TimedLaunch tl("k_reduce", s);
        k_reduce<<<1, SAMPLE_NT, 0, s>>>(w.partials, (int)grid.x, chi2);
    } else {
        TimedLaunch tl("k_sample_vis", s);
        k_sample<T, false><<<grid, SAMPLE_NT, 0, s>>>(XT, g, sa, o.u, o.v, nullptr, nullptr,
                                                      nullptr, (c2<T> *)vis, o.perm, w.partials,
                                                      w.ctl);
    }
    return check_launch();
}

}  // namespace gal

using namespace gal;

// ---------------------------------------------------------------------------
// datasets
struct gal_dataset {
    int precision;  // 8 or 4
    int device;
    int64_t M;
    double rho_max;
    void *buf;      // one allocation: u, v, re, im, w, perm (locality order)
    void *u, *v, *re, *im, *w;
    int32_t *perm;  // perm[k] = registration index of stored point k
};

// The definitions below take their C linkage from the declarations in the
// header; the helper templates between them are internal.

const char *gal_version(void) { return "galario-hip 0.1 (gfx950)"; }
const char *gal_last_error(void) { return t_err.c_str(); }

int gal_init(int device) {
    int n = 0;
    GAL_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(GAL_ERR_SIZE, "device %d of %d", device, n);
    return init_device(device);
}

size_t gal_workspace_bytes_d(int Nxy, int64_t M) {
    if (!pow2_in_range(Nxy) || M < 0) return 0;
    return ws_bytes<double>(Nxy, M);
}
size_t gal_workspace_bytes_f(int Nxy, int64_t M) {
    if (!pow2_in_range(Nxy) || M < 0) return 0;
    return ws_bytes<float>(Nxy, M);
}

int gal_workspace_init(void *ws, size_t ws_bytes_, void *stream) {
    if (!ws) return fail(GAL_ERR_NULL, "workspace is NULL");
    if (ws_bytes_ < 256) return fail(GAL_ERR_WORKSPACE, "workspace smaller than 256 bytes");
    hipStream_t s = (hipStream_t)stream;
    k_ctrl_zero<<<1, 64, 0, s>>>((Control *)ws);
    return check_launch();
}

int gal_read_status(void *ws, void *stream, int *status) {
    if (!ws || !status) return fail(GAL_ERR_NULL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    Control c;
    GAL_HIP(hipMemcpyAsync(&c, ws, sizeof(Control), hipMemcpyDeviceToHost, s));
    GAL_HIP(hipStreamSynchronize(s));
    *status = c.flag;
    if (c.flag) {
        k_ctrl_zero<<<1, 64, 0, s>>>((Control *)ws);
        int rc = check_launch();
        if (rc) return rc;
        GAL_HIP(hipStreamSynchronize(s));
    }
    return GAL_OK;
}

// ---- sweep --------------------------------------------------------------
template <typename T>
static int sweep_impl(const T *I, int Nr, double Rmin, double dR, int Nxy, double dxy, double inc,
                      T *image, void *stream) {
    if (!I || !image) return fail(GAL_ERR_NULL, "NULL array");
    int rc = check_image_scalars(Nxy, dxy, 0.0, 0.0, 0.0, inc);
    if (rc) return rc;
    rc = check_profile(Nr, Rmin, dR);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const SweepArgs sw = make_sweep(Nr, Rmin, dR, dxy, inc);
    const int64_t n = (int64_t)Nxy * Nxy;
    {
        TimedLaunch tl("k_sweep", s);
        k_sweep<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(I, sw, Nxy, image);
    }
    return check_launch();
}
int gal_sweep_d(const double *I, int Nr, double Rmin, double dR, int Nxy, double dxy, double inc,
                double *image, void *stream) {
    return sweep_impl<double>(I, Nr, Rmin, dR, Nxy, dxy, inc, image, stream);
}
int gal_sweep_f(const float *I, int Nr, double Rmin, double dR, int Nxy, double dxy, double inc,
                float *image, void *stream) {
    return sweep_impl<float>(I, Nr, Rmin, dR, Nxy, dxy, inc, image, stream);
}

// ---- raw-array calls -------------------------------------------------------
template <typename T>
static int image_call(const T *image, int Nxy, double dxy, const T *u, const T *v, const T *re,
                      const T *im, const T *w, int64_t M, double PA, double dRA, double dDec,
                      double inc, T *vis, double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!image || (M > 0 && (!u || !v))) return fail(GAL_ERR_NULL, "NULL array");
    if (chi2 && M > 0 && (!re || !im || !w)) return fail(GAL_ERR_NULL, "NULL observation array");
    if (!chi2 && M > 0 && !vis) return fail(GAL_ERR_NULL, "NULL output");
    if (M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);
    if (rc) return rc;
    const Geom g = geom_full(Nxy);
    return run_path<T>(image, false, SweepArgs{}, g, dxy, Obs<T>{u, v, re, im, w, M, nullptr}, PA, dRA, dDec,
                       inc, vis, chi2, ws, ws_bytes_, (hipStream_t)stream);
}

template <typename T>
static int profile_call(const T *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                        const T *u, const T *v, const T *re, const T *im, const T *w, int64_t M,
                        double inc, double PA, double dRA, double dDec, T *vis, double *chi2,
                        void *ws, size_t ws_bytes_, void *stream) {
    if (!I || (M > 0 && (!u || !v))) return fail(GAL_ERR_NULL, "NULL array");
    if (chi2 && M > 0 && (!re || !im || !w)) return fail(GAL_ERR_NULL, "NULL observation array");
    if (!chi2 && M > 0 && !vis) return fail(GAL_ERR_NULL, "NULL output");
    if (M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);
    if (rc) return rc;
    rc = check_profile(Nr, Rmin, dR);
    if (rc) return rc;
    const Geom g = geom_full(Nxy);
    return run_path<T>(I, true, make_sweep(Nr, Rmin, dR, dxy, inc), g, dxy,
                       Obs<T>{u, v, re, im, w, M, nullptr}, PA, dRA, dDec, 0.0, vis, chi2, ws, ws_bytes_,
                       (hipStream_t)stream);
}

int gal_sampleImage_d(const double *image, int Nxy, double dxy, const double *u, const double *v,
                      int64_t M, double PA, double dRA, double dDec, double inc, double *vis,
                      void *ws, size_t ws_bytes_, void *stream) {
    return image_call<double>(image, Nxy, dxy, u, v, nullptr, nullptr, nullptr, M, PA, dRA, dDec,
                              inc, vis, nullptr, ws, ws_bytes_, stream);
}
int gal_sampleImage_f(const float *image, int Nxy, double dxy, const float *u, const float *v,
                      int64_t M, double PA, double dRA, double dDec, double inc, float *vis,
                      void *ws, size_t ws_bytes_, void *stream) {
    return image_call<float>(image, Nxy, dxy, u, v, nullptr, nullptr, nullptr, M, PA, dRA, dDec,
                             inc, vis, nullptr, ws, ws_bytes_, stream);
}
int gal_sampleProfile_d(const double *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                        const double *u, const double *v, int64_t M, double inc, double PA,
                        double dRA, double dDec, double *vis, void *ws, size_t ws_bytes_,
                        void *stream) {
    return profile_call<double>(I, Nr, Rmin, dR, Nxy, dxy, u, v, nullptr, nullptr, nullptr, M, inc,
                                PA, dRA, dDec, vis, nullptr, ws, ws_bytes_, stream);
}
int gal_sampleProfile_f(const float *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                        const float *u, const float *v, int64_t M, double inc, double PA,
                        double dRA, double dDec, float *vis, void *ws, size_t ws_bytes_,
                        void *stream) {
    return profile_call<float>(I, Nr, Rmin, dR, Nxy, dxy, u, v, nullptr, nullptr, nullptr, M, inc,
                               PA, dRA, dDec, vis, nullptr, ws, ws_bytes_, stream);
}
int gal_chi2Image_d(const double *image, int Nxy, double dxy, const double *u, const double *v,
                    const double *re, const double *im, const double *w, int64_t M, double PA,
                    double dRA, double dDec, double inc, double *chi2, void *ws, size_t ws_bytes_,
                    void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return image_call<double>(image, Nxy, dxy, u, v, re, im, w, M, PA, dRA, dDec, inc, nullptr,
                              chi2, ws, ws_bytes_, stream);
}
int gal_chi2Image_f(const float *image, int Nxy, double dxy, const float *u, const float *v,
                    const float *re, const float *im, const float *w, int64_t M, double PA,
                    double dRA, double dDec, double inc, double *chi2, void *ws, size_t ws_bytes_,
                    void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return image_call<float>(image, Nxy, dxy, u, v, re, im, w, M, PA, dRA, dDec, inc, nullptr,
                             chi2, ws, ws_bytes_, stream);
}
int gal_chi2Profile_d(const double *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                      const double *u, const double *v, const double *re, const double *im,
                      const double *w, int64_t M, double inc, double PA, double dRA, double dDec,
                      double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return profile_call<double>(I, Nr, Rmin, dR, Nxy, dxy, u, v, re, im, w, M, inc, PA, dRA, dDec,
                                nullptr, chi2, ws, ws_bytes_, stream);
}
int gal_chi2Profile_f(const float *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                      const float *u, const float *v, const float *re, const float *im,
                      const float *w, int64_t M, double inc, double PA, double dRA, double dDec,
                      double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return profile_call<float>(I, Nr, Rmin, dR, Nxy, dxy, u, v, re, im, w, M, inc, PA, dRA, dDec,
                               nullptr, chi2, ws, ws_bytes_, stream);
}

// ---- separately callable steps -------------------------------------------
template <typename T>
static int spectrum_impl(const T *image, int Nxy, T *spec, void *ws, size_t ws_bytes_,
                         void *stream) {
    if (!image || !spec) return fail(GAL_ERR_NULL, "NULL array");
    if (!pow2_in_range(Nxy)) return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", Nxy);
    int rc = ensure_init();
    if (rc) return rc;
    WS w;
    rc = carve<T>(ws, ws_bytes_, Nxy, 0, w);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Geom g = geom_full(Nxy);
    c2<T> *XT = (c2<T> *)w.xt;
    rc = dispatch_fft<T>(Nxy, image, false, SweepArgs{}, g, XT, s);
    if (rc) return rc;
    const int64_t n = (int64_t)Nxy * (Nxy / 2 + 1);
    {
        TimedLaunch tl("k_spec_out", s);
        k_spec_out<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(XT, g, (c2<T> *)spec);
    }
    return check_launch();
}
int gal_spectrum_d(const double *image, int Nxy, double *spec, void *ws, size_t ws_bytes_,
                   void *stream) {
    return spectrum_impl<double>(image, Nxy, spec, ws, ws_bytes_, stream);
}
int gal_spectrum_f(const float *image, int Nxy, float *spec, void *ws, size_t ws_bytes_,
                   void *stream) {
    return spectrum_impl<float>(image, Nxy, spec, ws, ws_bytes_, stream);
}

template <typename T>
static int sample_spectrum_impl(const T *spec, int Nxy, double dxy, const T *u, const T *v,
                                int64_t M, double PA, double dRA, double dDec, double inc, T *vis,
                                void *ws, size_t ws_bytes_, void *stream) {
    if (!spec || (M > 0 && (!u || !v || !vis))) return fail(GAL_ERR_NULL, "NULL array");
    if (M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);
    if (rc) return rc;
    WS w;
    rc = carve<T>(ws, ws_bytes_, Nxy, M, w);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Geom g = geom_full(Nxy);
    c2<T> *XT = (c2<T> *)w.xt;
    const int64_t n = (int64_t)(Nxy / 2 + 1) * (2 * g.P + 1);
    {
        TimedLaunch tl("k_spec_in", s);
        k_spec_in<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const c2<T> *)spec, g, XT);
    }
    rc = check_launch();
    if (rc) return rc;
    const SampleArgs sa = make_sample(g, M, dxy, PA, dRA, dDec, inc);
    {
        TimedLaunch tl("k_sample_vis", s);
        k_sample<T, false><<<(unsigned)sample_blocks(M), SAMPLE_NT, 0, s>>>(
            XT, g, sa, u, v, nullptr, nullptr, nullptr, (c2<T> *)vis, nullptr, w.partials, w.ctl);
    }
    return check_launch();
}
int gal_sample_spectrum_d(const double *spec, int Nxy, double dxy, const double *u, const double *v,
                          int64_t M, double PA, double dRA, double dDec, double inc, double *vis,
                          void *ws, size_t ws_bytes_, void *stream) {
    return sample_spectrum_impl<double>(spec, Nxy, dxy, u, v, M, PA, dRA, dDec, inc, vis, ws,
                                        ws_bytes_, stream);
}
int gal_sample_spectrum_f(const float *spec, int Nxy, double dxy, const float *u, const float *v,
                          int64_t M, double PA, double dRA, double dDec, double inc, float *vis,
                          void *ws, size_t ws_bytes_, void *stream) {
    return sample_spectrum_impl<float>(spec, Nxy, dxy, u, v, M, PA, dRA, dDec, inc, vis, ws,
                                       ws_bytes_, stream);
}

// ---- datasets -------------------------------------------------------------
// Morton (Z-order) key of a uv point on a 2^16 x 2^16 grid over
// [-rho_max, rho_max]^2: neighbouring keys are neighbouring points, and a
// rotation by PA keeps neighbours together, so a wavefront of consecutive
// points gathers from a few cache lines of the spectrum.
static uint32_t spread16(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

static uint32_t morton_key(double u, double v, double rho_max) {
    const double sc = rho_max > 0.0 ? 32767.5 / rho_max : 0.0;
    double x = (u * sc) + 32767.5, y = (v * sc) + 32767.5;
    x = x < 0.0 ? 0.0 : (x > 65535.0 ? 65535.0 : x);
    y = y < 0.0 ? 0.0 : (y > 65535.0 ? 65535.0 : y);
    return spread16((uint32_t)x) | (spread16((uint32_t)y) << 1);
}

template <typename T>
static int dataset_create(const T *u, const T *v, const T *re, const T *im, const T *w, int64_t M,
                          void *stream, gal_dataset **out) {
    if (!out) return fail(GAL_ERR_NULL, "NULL out");
    *out = nullptr;
    if (M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    if (M > (int64_t)0x7fffffff) return fail(GAL_ERR_SIZE, "M above 2^31 - 1");
    if (M > 0 && (!u || !v)) return fail(GAL_ERR_NULL, "NULL u or v");
    const bool has_obs = re && im && w;
    if ((re || im || w) && !has_obs) return fail(GAL_ERR_NULL, "re, im, w: give all or none");
    int rc = ensure_init();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int n_cols = has_obs ? 5 : 2;
    const T *src[5] = {u, v, re, im, w};
    // observations to the host, in registration order
    std::vector<std::vector<T>> h(n_cols, std::vector<T>((size_t)M));
    for (int c = 0; c < n_cols && M > 0; ++c)
        GAL_HIP(hipMemcpyAsync(h[c].data(), src[c], (size_t)M * sizeof(T), hipMemcpyDeviceToHost, s));
    GAL_HIP(hipStreamSynchronize(s));
    double r2max = 0.0;
    for (int64_t k = 0; k < M; ++k) {
        const double uu = h[0][k], vv = h[1][k];
        const double r2 = uu * uu + vv * vv;
        if (!std::isfinite(r2)) return fail(GAL_ERR_SCALAR, "non-finite uv coordinate at %lld",
                                            (long long)k);
        r2max = r2 > r2max ? r2 : r2max;
    }
    const double rho_max = std::sqrt(r2max);
    // locality order
    std::vector<std::pair<uint32_t, int32_t>> key((size_t)M);
    for (int64_t k = 0; k < M; ++k)
        key[k] = {morton_key((double)h[0][k], (double)h[1][k], rho_max), (int32_t)k};
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint32_t, int32_t> &a, const std::pair<uint32_t, int32_t> &b) {
                         return a.first < b.first;
                     });
    std::vector<int32_t> perm((size_t)M);
    for (int64_t k = 0; k < M; ++k) perm[k] = key[k].second;
    std::vector<T> tmp((size_t)M);
    for (int c = 0; c < n_cols; ++c) {
        for (int64_t k = 0; k < M; ++k) tmp[k] = h[c][perm[k]];
        h[c].swap(tmp);
    }

    gal_dataset *ds = new gal_dataset();
    ds->precision = (int)sizeof(T);
    GAL_HIP(hipGetDevice(&ds->device));
    ds->M = M;
    ds->rho_max = rho_max;
    const size_t col = align256((size_t)(M > 0 ? M : 1) * sizeof(T));
    const size_t pcol = align256((size_t)(M > 0 ? M : 1) * sizeof(int32_t));
    if (hipMalloc(&ds->buf, col * n_cols + pcol) != hipSuccess) {
        delete ds;
        return fail(GAL_ERR_WORKSPACE, "out of device memory for a dataset of %lld points",
                    (long long)M);
    }
    char *p = (char *)ds->buf;
    void *dst[5] = {p, p + col, p + 2 * col, p + 3 * col, p + 4 * col};
    ds->u = dst[0];
    ds->v = dst[1];
    ds->re = has_obs ? dst[2] : nullptr;
    ds->im = has_obs ? dst[3] : nullptr;
    ds->w = has_obs ? dst[4] : nullptr;
    ds->perm = (int32_t *)(p + col * n_cols);
    bool ok = true;
    for (int c = 0; c < n_cols && M > 0; ++c)
        ok = ok && hipMemcpyAsync(dst[c], h[c].data(), (size_t)M * sizeof(T),
                                  hipMemcpyHostToDevice, s) == hipSuccess;
    if (M > 0)
        ok = ok && hipMemcpyAsync(ds->perm, perm.data(), (size_t)M * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        (void)hipFree(ds->buf);
        delete ds;
        return fail(GAL_ERR_HIP, "dataset upload failed");
    }
    *out = ds;
    return GAL_OK;
}

int gal_dataset_create_d(const double *u, const double *v, const double *re, const double *im,
                         const double *w, int64_t M, void *stream, gal_dataset **out) {
    return dataset_create<double>(u, v, re, im, w, M, stream, out);
}
int gal_dataset_create_f(const float *u, const float *v, const float *re, const float *im,
                         const float *w, int64_t M, void *stream, gal_dataset **out) {
    return dataset_create<float>(u, v, re, im, w, M, stream, out);
}
int gal_dataset_destroy(gal_dataset *ds) {
    if (!ds) return GAL_OK;
    int cur = 0;
    GAL_HIP(hipGetDevice(&cur));
    if (cur != ds->device) GAL_HIP(hipSetDevice(ds->device));
    hipError_t e = hipFree(ds->buf);
    if (cur != ds->device) (void)hipSetDevice(cur);
    delete ds;
    if (e != hipSuccess) return fail(GAL_ERR_HIP, "hipFree: %s", hipGetErrorString(e));
    return GAL_OK;
}
int gal_dataset_info(const gal_dataset *ds, int64_t *M, double *rho_max, int *precision) {
    if (!ds) return fail(GAL_ERR_NULL, "NULL dataset");
    if (M) *M = ds->M;
    if (rho_max) *rho_max = ds->rho_max;
    if (precision) *precision = ds->precision;
    return GAL_OK;
}

int gal_dataset_geometry(const gal_dataset *ds, int Nxy, double dxy, int *Q, int *P) {
    if (!ds || !Q || !P) return fail(GAL_ERR_NULL, "NULL argument");
    int rc = check_image_scalars(Nxy, dxy, 0.0, 0.0, 0.0, 0.0);
    if (rc) return rc;
    const Geom g = geom_pruned(Nxy, dxy, ds->rho_max);
    *Q = g.Q;
    *P = g.P;
    return GAL_OK;
}

template <typename T>
static int ds_call(const gal_dataset *ds, const T *src, bool profile, int Nr, double Rmin,
                   double dR, int Nxy, double dxy, double inc, double PA, double dRA, double dDec,
                   T *vis, double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!ds || !src) return fail(GAL_ERR_NULL, "NULL argument");
    if (ds->precision != (int)sizeof(T))
        return fail(GAL_ERR_UNSUPPORTED, "dataset precision %d differs from the call", ds->precision);
    if (chi2 && !ds->re) return fail(GAL_ERR_UNSUPPORTED, "dataset holds no observations");
    if (!chi2 && ds->M > 0 && !vis) return fail(GAL_ERR_NULL, "NULL output");
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);
    if (rc) return rc;
    if (profile) {
        rc = check_profile(Nr, Rmin, dR);
        if (rc) return rc;
    }
    const double du = 1.0 / ((double)Nxy * dxy);
    if (!(ds->rho_max < ((double)(Nxy / 2) - 1.0) * du))
        return fail(GAL_ERR_UV_RANGE,
                    "rho_max = %.6g lambda reaches beyond the half spectrum (limit %.6g for "
                    "Nxy=%d, dxy=%.6g)",
                    ds->rho_max, ((double)(Nxy / 2) - 1.0) * du, Nxy, dxy);
    const Geom g = geom_pruned(Nxy, dxy, ds->rho_max);
    const Obs<T> o{(const T *)ds->u, (const T *)ds->v, (const T *)ds->re, (const T *)ds->im,
                   (const T *)ds->w, ds->M, ds->perm};
    const SweepArgs sw = profile ? make_sweep(Nr, Rmin, dR, dxy, inc) : SweepArgs{};
    return run_path<T>(src, profile, sw, g, dxy, o, PA, dRA, dDec, profile ? 0.0 : inc, vis, chi2,
                       ws, ws_bytes_, (hipStream_t)stream);
}

int gal_chi2Image_ds_d(const gal_dataset *ds, const double *image, int Nxy, double dxy, double PA,
                       double dRA, double dDec, double inc, double *chi2, void *ws,
                       size_t ws_bytes_, void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return ds_call<double>(ds, image, false, 0, 0, 0, Nxy, dxy, inc, PA, dRA, dDec, nullptr, chi2,
                           ws, ws_bytes_, stream);
}
int gal_chi2Image_ds_f(const gal_dataset *ds, const float *image, int Nxy, double dxy, double PA,
                       double dRA, double dDec, double inc, double *chi2, void *ws,
                       size_t ws_bytes_, void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return ds_call<float>(ds, image, false, 0, 0, 0, Nxy, dxy, inc, PA, dRA, dDec, nullptr, chi2, ws,
                          ws_bytes_, stream);
}
int gal_chi2Profile_ds_d(const gal_dataset *ds, const double *I, int Nr, double Rmin, double dR,
                         int Nxy, double dxy, double inc, double PA, double dRA, double dDec,
                         double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return ds_call<double>(ds, I, true, Nr, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec, nullptr, chi2,
                           ws, ws_bytes_, stream);
}
int gal_chi2Profile_ds_f(const gal_dataset *ds, const float *I, int Nr, double Rmin, double dR,
                         int Nxy, double dxy, double inc, double PA, double dRA, double dDec,
                         double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!chi2) return fail(GAL_ERR_NULL, "NULL chi2");
    return ds_call<float>(ds, I, true, Nr, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec, nullptr, chi2,
                          ws, ws_bytes_, stream);
}
int gal_sampleImage_ds_d(const gal_dataset *ds, const double *image, int Nxy, double dxy,
                         double PA, double dRA, double dDec, double inc, double *vis, void *ws,
                         size_t ws_bytes_, void *stream) {
    return ds_call<double>(ds, image, false, 0, 0, 0, Nxy, dxy, inc, PA, dRA, dDec, vis, nullptr,
                           ws, ws_bytes_, stream);
}
int gal_sampleImage_ds_f(const gal_dataset *ds, const float *image, int Nxy, double dxy,
                         double PA, double dRA, double dDec, double inc, float *vis, void *ws,
                         size_t ws_bytes_, void *stream) {
    return ds_call<float>(ds, image, false, 0, 0, 0, Nxy, dxy, inc, PA, dRA, dDec, vis, nullptr, ws,
                          ws_bytes_, stream);
}
int gal_sampleProfile_ds_d(const gal_dataset *ds, const double *I, int Nr, double Rmin, double dR,
                           int Nxy, double dxy, double inc, double PA, double dRA, double dDec,
                           double *vis, void *ws, size_t ws_bytes_, void *stream) {
    return ds_call<double>(ds, I, true, Nr, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec, vis, nullptr,
                           ws, ws_bytes_, stream);
}
int gal_sampleProfile_ds_f(const gal_dataset *ds, const float *I, int Nr, double Rmin, double dR,
                           int Nxy, double dxy, double inc, double PA, double dRA, double dDec,
                           float *vis, void *ws, size_t ws_bytes_, void *stream) {
    return ds_call<float>(ds, I, true, Nr, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec, vis, nullptr, ws,
                          ws_bytes_, stream);
}

// ---- timing ---------------------------------------------------------------
int gal_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm_on = on != 0;
    return GAL_OK;
}

int gal_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    for (auto &r : g_tm_recs) {
        g_tm_pool.push_back(r.a);
        g_tm_pool.push_back(r.b);
    }
    g_tm_recs.clear();
    return GAL_OK;
}

int gal_timing_read(int cap, const char **names, double *total_ms, int64_t *launches) {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    std::vector<const char *> nm;
    std::vector<double> ms;
    std::vector<int64_t> cnt;
    for (auto &r : g_tm_recs) {
        GAL_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        GAL_HIP(hipEventElapsedTime(&t, r.a, r.b));
        size_t k = 0;
        while (k < nm.size() && std::strcmp(nm[k], r.name) != 0) ++k;
        if (k == nm.size()) {
            nm.push_back(r.name);
            ms.push_back(0.0);
            cnt.push_back(0);
        }
        ms[k] += t;
        cnt[k] += 1;
    }
    for (size_t k = 0; k < nm.size() && (int)k < cap; ++k) {
        if (names) names[k] = nm[k];
        if (total_ms) total_ms[k] = ms[k];
        if (launches) launches[k] = cnt[k];
    }
    return (int)nm.size();
}
