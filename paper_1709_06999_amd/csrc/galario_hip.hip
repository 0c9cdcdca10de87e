// galario_hip.hip -- host side of the C ABI declared in include/galario_hip.h.
//
// Argument checks, the choice of which part of the half spectrum to
// transform, workspace carving, kernel launches and per-kernel timing.  All
// arithmetic of the path runs in the kernels of kernels.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <utility>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/galario_hip.h"
#include "adjoint.h"
#include "batch.h"
#include "geograd.h"
#include "kernels.h"
#include "mixed_radix.h"

namespace gal {

__device__ c2<double> g_tw_d[2 * TW_MAX];
__device__ c2<float> g_tw_f[2 * TW_MAX];

// Workspace of gal_chi2Profile_ds_scratch_d, for callers that cannot allocate.
// Each device holds its own copy; host code uses only the per-device address
// that hipGetSymbolAddress returns (g_scratch_ptr), never the array's name.
__device__ __align__(256) char scratch[GAL_SCRATCH_BYTES];

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
static std::vector<void *> g_scratch_ptr;  // per device: device address of `scratch`

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
    // the scratch workspace: its address on this device, and its control
    // block (status flag) cleared once, as gal_workspace_init does for a
    // caller's workspace
    void *sp = nullptr;
    GAL_HIP(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
    GAL_HIP(hipMemset(sp, 0, 256));
    GAL_HIP(hipDeviceSynchronize());
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    g_scratch_ptr[dev] = sp;
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
// kernel launches, with per-kernel timing from the dispatch's own start / end
// timestamps (hipExtLaunchKernelGGL) when timing is enabled
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

static bool tm_begin(hipEvent_t &a, hipEvent_t &b) {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    if (!g_tm_on) return false;
    a = tm_event();
    b = tm_event();
    return a && b;
}

static void tm_end(const char *name, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm_recs.push_back({name, a, b});
}

static int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GAL_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return GAL_OK;
}

// Every argument is converted to the kernel's parameter type before launch
// (pointers by a plain cast: the buffers are reused with several layouts).
template <typename K, typename A>
static inline K arg_cast(A &&a) {
    if constexpr (std::is_pointer<K>::value) return (K)(a);
    else return static_cast<K>(a);
}

template <typename... KArgs, typename... Args>
static int launch_sm(const char *name, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                     unsigned shmem, hipStream_t s, Args &&...args) {
    static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
    if (grid.x == 0 || grid.y == 0) return GAL_OK;
    hipEvent_t a = nullptr, b = nullptr;
    if (tm_begin(a, b)) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0, arg_cast<KArgs>(args)...);
        tm_end(name, a, b);
    } else {
        kernel<<<grid, block, shmem, s>>>(arg_cast<KArgs>(args)...);
    }
    return check_launch();
}

template <typename... KArgs, typename... Args>
static int launch(const char *name, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                  hipStream_t s, Args &&...args) {
    return launch_sm(name, kernel, grid, block, 0u, s, static_cast<Args &&>(args)...);
}

// ---------------------------------------------------------------------------
// FFT shapes.  Each pass kernel exists in up to three variants that differ
// in the values each thread holds (E = 16, 8, 4: fewer values = more
// threads per transform, more waves in flight, more radix-E passes).  The
// autotuner (gal_autotune_*) times them per image size and precision; the
// defaults below are used until it has run.
enum FftKind { K_ROWS_IMG = 0, K_COLS = 1, K_ROWS_SYM = 2, K_COLS_SYM = 3, NKIND = 4 };
constexpr int NVAR = 3;
constexpr int var_E(int var) { return var == 0 ? 16 : (var == 1 ? 8 : 4); }
constexpr int min_c(int a, int b) { return a < b ? a : b; }
constexpr int max_c(int a, int b) { return a > b ? a : b; }

// rows of a general image: B rows of length N/2 per block (B >= 4 where the
// LDS allows, so that the transposed store writes >= 64-byte runs)
constexpr int rows_B(int N) {
    return N >= 8192 ? 1 : (N >= 4096 ? 2 : min_c(N, max_c(4, 2048 / N)));
}
// complex length-N passes (columns, swept-profile row pairs): B sequences
constexpr int cols_B(int N) { return max_c(1, 1024 / N); }
// threads for B sequences of length L with E values each, capped at 1024
constexpr int shape_E(int B, int L, int E) {
    return (B * L / E > 1024) ? (B * L / 1024) : (E > B * L ? B * L : E);
}

template <typename T, int L, int B, int E>
using CfgE = FFTCfg<T, L, B, B * L / shape_E(B, L, E), min_c(16, min_c(shape_E(B, L, E), L))>;

template <typename T>
struct FftJob {
    const T *src;    // image (rows_image) or profile (rows_sym)
    SweepArgs sw;
    Geom g;
    int Qe;          // even column count (swept-profile passes)
    void *buf;       // intermediate / spectrum
    hipStream_t s;
    void *buf2 = nullptr;  // spectrum of a column pass that cannot run in place
};
template <typename T>
using FftFn = int (*)(const FftJob<T> &);

template <typename T, int N, int VAR>
static int run_rows_img(const FftJob<T> &j) {
    constexpr int B = rows_B(N);
    using C = CfgE<T, N / 2, B, var_E(VAR)>;
    return launch("k_rows_image", k_rows<T, C, false>, dim3(N / B), dim3(C::NT), j.s, j.src, j.sw,
                  j.g, j.buf);
}
template <typename T, int N, int VAR>
static int run_cols(const FftJob<T> &j) {
    constexpr int B = cols_B(N);
    using C = CfgE<T, N, B, var_E(VAR)>;
    return launch("k_cols", k_cols<T, C>, dim3((j.g.Q + B - 1) / B), dim3(C::NT), j.s, j.g, j.buf);
}
// rows of a swept profile: variant 1 transforms each row pair at full length
// (rows_sym_body, E = 8); variants 0 and 2 use the half-length transform of
// even rows (rows_even_body, E = 8 and 4)
template <typename T, int N, int VAR>
static int run_rows_sym(const FftJob<T> &j) {
    constexpr int B = cols_B(N);
    const int pairs = N / 4 + 1;
    if constexpr (VAR == 1) {
        using C = CfgE<T, N, B, 8>;
        return launch("k_rows_sym", k_rows_sym<T, C>, dim3((pairs + B - 1) / B), dim3(C::NT), j.s,
                      j.src, j.sw, j.g, j.Qe, j.buf);
    } else {
        using C = CfgE<T, N / 2, B, VAR == 0 ? 8 : 4>;
        return launch("k_rows_even", k_rows_even<T, C>, dim3((pairs + B - 1) / B), dim3(C::NT),
                      j.s, j.src, j.sw, j.g, j.Qe, j.buf);
    }
}
// columns of a swept profile: variant 0 takes the half-length transform of
// the even columns (cols_even_body, E = 8), variants 1 and 2 the full-length
// one (cols_sym_body, E = 8 and 4)
template <typename T, int N, int VAR>
static int run_cols_sym(const FftJob<T> &j) {
    constexpr int B = cols_B(N);
    const int pairs = j.Qe / 2;
    if constexpr (VAR == 0) {
        using C = CfgE<T, N / 2, B, 8>;
        return launch("k_cols_even", k_cols_even<T, C>, dim3((pairs + B - 1) / B), dim3(C::NT),
                      j.s, j.g, j.Qe, j.buf);
    } else {
        using C = CfgE<T, N, B, var_E(VAR)>;
        return launch("k_cols_sym", k_cols_sym<T, C>, dim3((pairs + B - 1) / B), dim3(C::NT),
                      j.s, j.g, j.Qe, j.buf);
    }
}

// 16384^2: one schedule per pass.  Rows of images at half length (E = 8);
// swept profiles by the half-length transform of even sequences in both
// passes; image columns in LDS in FP32, in two launches (four-step) in FP64,
// whose column of 256 KB does not fit.
constexpr int NXY_BIG = 16384;
template <typename T>
constexpr bool four_step(int N) { return N == NXY_BIG && sizeof(T) == 8; }

template <typename T>
static int run_cols_even_big(const FftJob<T> &j) {
    using C = CfgE<T, NXY_BIG / 2, 1, 8>;
    return launch("k_cols_even", k_cols_even<T, C>, dim3(j.Qe / 2), dim3(C::NT), j.s, j.g, j.Qe,
                  j.buf);
}
template <typename T>
static int run_cols4_big(const FftJob<T> &j) {
    constexpr int N1 = 128, B = 16;
    static_assert(N1 * N1 == NXY_BIG, "four-step factors");
    using C = CfgE<T, N1, B, 8>;
    if (!j.buf2) return fail(GAL_ERR_WORKSPACE, "no spectrum buffer for the 16384 column pass");
    int rc = launch("k_cols4a", k_cols4a<T, C, NXY_BIG>, dim3(N1 / B, j.g.Q), dim3(C::NT), j.s,
                    j.g, j.buf);
    if (rc) return rc;
    return launch("k_cols4b", k_cols4b<T, C, NXY_BIG>, dim3(N1 / B, j.g.Q), dim3(C::NT), j.s, j.g,
                  j.buf, j.buf2, 2 * j.g.P + 1);
}
template <typename T>
static FftFn<T> fft_fn_big(int kind) {
    switch (kind) {
        case K_ROWS_IMG: return run_rows_img<T, NXY_BIG, 1>;
        case K_COLS:
            if constexpr (four_step<T>(NXY_BIG)) return run_cols4_big<T>;
            else return run_cols<T, NXY_BIG, 0>;
        case K_ROWS_SYM: return run_rows_sym<T, NXY_BIG, 0>;
        default: return run_cols_even_big<T>;
    }
}

// variant table [log2 N - 4][kind][var]; small images compile one variant
template <typename T, int N>
struct VarTable {
    static constexpr bool many = N >= 256;
    static FftFn<T> get(int kind, int var) {
        if (!many) var = 0;
        switch (kind) {
            case K_ROWS_IMG:
                return var == 0 ? run_rows_img<T, N, 0>
                                : (var == 1 ? run_rows_img<T, N, (many ? 1 : 0)>
                                            : run_rows_img<T, N, (many ? 2 : 0)>);
            case K_COLS:
                return var == 0 ? run_cols<T, N, 0>
                                : (var == 1 ? run_cols<T, N, (many ? 1 : 0)>
                                            : run_cols<T, N, (many ? 2 : 0)>);
            case K_ROWS_SYM:
                return var == 0 ? run_rows_sym<T, N, 0>
                                : (var == 1 ? run_rows_sym<T, N, (many ? 1 : 0)>
                                            : run_rows_sym<T, N, (many ? 2 : 0)>);
            default:
                return var == 0 ? run_cols_sym<T, N, 0>
                                : (var == 1 ? run_cols_sym<T, N, (many ? 1 : 0)>
                                            : run_cols_sym<T, N, (many ? 2 : 0)>);
        }
    }
};

template <typename T>
static FftFn<T> fft_fn(int N, int kind, int var) {
    switch (N) {
        case 16: return VarTable<T, 16>::get(kind, var);
        case 32: return VarTable<T, 32>::get(kind, var);
        case 64: return VarTable<T, 64>::get(kind, var);
        case 128: return VarTable<T, 128>::get(kind, var);
        case 256: return VarTable<T, 256>::get(kind, var);
        case 512: return VarTable<T, 512>::get(kind, var);
        case 1024: return VarTable<T, 1024>::get(kind, var);
        case 2048: return VarTable<T, 2048>::get(kind, var);
        case 4096: return VarTable<T, 4096>::get(kind, var);
        case 8192: return VarTable<T, 8192>::get(kind, var);
        default: return nullptr;
    }
}

static int log2i(int N) {
    int l = 0;
    while ((1 << l) < N) ++l;
    return l;
}

// chosen variant per [precision 0 = double, 1 = float][log2 N][kind]; -1 = default
static std::mutex g_tune_mu;
static int g_choice[2][14][NKIND];
static bool g_choice_init = false;

static int default_var(int N, int kind) {
    if (N < 256) return 0;
    return (kind == K_ROWS_IMG) ? 0 : 1;
}

template <typename T>
static int chosen_var(int N, int kind) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_choice_init) {
        for (auto &a : g_choice)
            for (auto &b : a)
                for (int &c : b) c = -1;
        g_choice_init = true;
    }
    const int v = g_choice[sizeof(T) == 8 ? 0 : 1][log2i(N)][kind];
    return v >= 0 ? v : default_var(N, kind);
}

template <typename T>
static int run_fft(int kind, const FftJob<T> &j) {
    if (j.g.N == NXY_BIG) return fft_fn_big<T>(kind)(j);
    FftFn<T> f = fft_fn<T>(j.g.N, kind, chosen_var<T>(j.g.N, kind));
    if (!f) return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", j.g.N);
    return f(j);
}

// ---------------------------------------------------------------------------
// batched FFT passes: one launch per (precision, kind, image size) group,
// blockIdx.y = job of the group
struct FftJobB {
    const JobDesc *jobs;
    const int *list;
    int count;
    int maxQ, maxQe;
    char *ws;
    hipStream_t s;
};
using FftFnB = int (*)(const FftJobB &);

template <typename T, int N, int VAR>
static int runb_rows_img(const FftJobB &j) {
    constexpr int B = rows_B(N);
    using C = CfgE<T, N / 2, B, var_E(VAR)>;
    return launch("kb_rows_image", kb_rows_img<T, C>, dim3(N / B, j.count), dim3(C::NT), j.s,
                  j.jobs, j.list, j.ws);
}
template <typename T, int N, int VAR>
static int runb_cols(const FftJobB &j) {
    constexpr int B = cols_B(N);
    using C = CfgE<T, N, B, var_E(VAR)>;
    return launch("kb_cols", kb_cols<T, C>, dim3((j.maxQ + B - 1) / B, j.count), dim3(C::NT), j.s,
                  j.jobs, j.list, j.ws);
}
template <typename T, int N, int VAR>
static int runb_rows_sym(const FftJobB &j) {
    constexpr int B = cols_B(N);
    if constexpr (VAR == 1) {
        using C = CfgE<T, N, B, 8>;
        return launch("kb_rows_sym", kb_rows_sym<T, C>, dim3((N / 4 + 1 + B - 1) / B, j.count),
                      dim3(C::NT), j.s, j.jobs, j.list, j.ws);
    } else {
        using C = CfgE<T, N / 2, B, VAR == 0 ? 8 : 4>;
        return launch("kb_rows_even", kb_rows_even<T, C>, dim3((N / 4 + 1 + B - 1) / B, j.count),
                      dim3(C::NT), j.s, j.jobs, j.list, j.ws);
    }
}
template <typename T, int N, int VAR>
static int runb_cols_sym(const FftJobB &j) {
    constexpr int B = cols_B(N);
    if constexpr (VAR == 0) {
        using C = CfgE<T, N / 2, B, 8>;
        return launch("kb_cols_even", kb_cols_even<T, C>, dim3((j.maxQe / 2 + B - 1) / B, j.count),
                      dim3(C::NT), j.s, j.jobs, j.list, j.ws);
    } else {
        using C = CfgE<T, N, B, var_E(VAR)>;
        return launch("kb_cols_sym", kb_cols_sym<T, C>, dim3((j.maxQe / 2 + B - 1) / B, j.count),
                      dim3(C::NT), j.s, j.jobs, j.list, j.ws);
    }
}

template <typename T, int N>
struct VarTableB {
    static constexpr bool many = N >= 256;
    template <int V>
    static FftFnB pick(int kind) {
        switch (kind) {
            case K_ROWS_IMG: return runb_rows_img<T, N, V>;
            case K_COLS: return runb_cols<T, N, V>;
            case K_ROWS_SYM: return runb_rows_sym<T, N, V>;
            default: return runb_cols_sym<T, N, V>;
        }
    }
    static FftFnB get(int kind, int var) {
        if (!many || var == 0) return pick<0>(kind);
        return var == 1 ? pick<(many ? 1 : 0)>(kind) : pick<(many ? 2 : 0)>(kind);
    }
};

template <typename T>
static FftFnB fft_fn_b(int N, int kind, int var) {
    switch (N) {
        case 16: return VarTableB<T, 16>::get(kind, var);
        case 32: return VarTableB<T, 32>::get(kind, var);
        case 64: return VarTableB<T, 64>::get(kind, var);
        case 128: return VarTableB<T, 128>::get(kind, var);
        case 256: return VarTableB<T, 256>::get(kind, var);
        case 512: return VarTableB<T, 512>::get(kind, var);
        case 1024: return VarTableB<T, 1024>::get(kind, var);
        case 2048: return VarTableB<T, 2048>::get(kind, var);
        case 4096: return VarTableB<T, 4096>::get(kind, var);
        case 8192: return VarTableB<T, 8192>::get(kind, var);
        default: return nullptr;
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

// [control 256 B][partials][XT][spectrum of a four-step column pass]
template <typename T>
static size_t spec2_bytes(int N) {
    return four_step<T>(N) ? align256((size_t)(N / 2 + 1) * (size_t)(N + 1) * sizeof(c2<T>)) : 0;
}

// mixed-radix sizes: the twiddle table of N and the swept image of a profile
template <typename T>
static size_t mr_bytes(int N) {
    if ((N & (N - 1)) == 0) return 0;
    return align256((size_t)N * sizeof(c2<T>)) + align256((size_t)N * (size_t)N * sizeof(T));
}

template <typename T>
static size_t ws_bytes(int N, int64_t M) {
    const size_t partials = align256((size_t)sample_blocks(M) * sizeof(double));
    const size_t xt = align256((size_t)(N / 2 + 1) * (size_t)(N + 2) * sizeof(c2<T>));
    return 256 + partials + xt + spec2_bytes<T>(N) + mr_bytes<T>(N);
}

struct WS {
    Control *ctl;
    double *partials;
    void *xt;
    void *spec2;  // four-step column pass output (NULL otherwise)
    void *mr;     // mixed-radix sizes: twiddle table, then the swept image (NULL otherwise)
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
    char *after_xt = (char *)out.xt + align256((size_t)(N / 2 + 1) * (size_t)(N + 2) * sizeof(c2<T>));
    out.spec2 = four_step<T>(N) ? after_xt : nullptr;
    out.mr = mr_bytes<T>(N) ? after_xt + spec2_bytes<T>(N) : nullptr;
    return GAL_OK;
}

// ---------------------------------------------------------------------------
// argument checks
// image sizes: powers of two from 16 to NXY_BIG for the forward calls (sweep,
// sample*, chi2*, datasets); up to 8192 for gradients, geometry gradients,
// batches, the autotuner and the separate spectrum calls
static bool pow2_upto(int N, int nmax) { return N >= 16 && N <= nmax && (N & (N - 1)) == 0; }
static bool pow2_in_range(int N) { return pow2_upto(N, 8192); }
// the forward calls also take even N = 2^a 3^b 5^c (not a power of two) in
// [16, 8192], on the mixed-radix path
static bool mr_size(int N) {
    if (N < 16 || N > MR_LMAX || (N & 1) || (N & (N - 1)) == 0) return false;
    int n = N;
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}
static bool fwd_size(int N) { return pow2_upto(N, NXY_BIG) || mr_size(N); }

// radices of a length-L transform (4s, then a 2, 3s, 5s); false if some pass
// would hold more than MR_BPT butterflies per thread of an NT-thread block
static bool mr_plan(int L, int N, int NT, MrPlan &pl) {
    pl.L = L;
    pl.tstride = N / L;
    pl.np = 0;
    int n = L;
    auto add = [&](int r) {
        if (pl.np >= MR_MAXPASS || L / r > MR_BPT * NT) return false;
        pl.radix[pl.np++] = r;
        n /= r;
        return true;
    };
    while (n % 4 == 0)
        if (!add(4)) return false;
    while (n % 2 == 0)
        if (!add(2)) return false;
    while (n % 3 == 0)
        if (!add(3)) return false;
    while (n % 5 == 0)
        if (!add(5)) return false;
    return n == 1;
}
// smallest pixel size: squared pixel radii stay far above the range where the
// sweep's square root would need scaling
constexpr double DXY_MIN = 1e-100;

// forward: the paper's calls (powers of two to NXY_BIG, mixed-radix sizes);
// otherwise powers of two to 8192
static int check_image_scalars(int N, double dxy, double PA, double dRA, double dDec, double inc,
                               bool forward = false) {
    if (forward && !fwd_size(N))
        return fail(GAL_ERR_SIZE,
                    "Nxy=%d: need a power of two in [16, %d] or an even 2^a 3^b 5^c in [16, %d]",
                    N, NXY_BIG, MR_LMAX);
    if (!forward && !pow2_in_range(N))
        return fail(GAL_ERR_SIZE, "Nxy=%d: need a power of two in [16, 8192] here", N);
    if (!(dxy >= DXY_MIN) || !std::isfinite(dxy)) return fail(GAL_ERR_SCALAR, "dxy must be >= 1e-100");
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
    a.tan_inc = std::tan(inc);
    a.dxs = dxy * a.inv_cos;
    a.t0 = -Rmin * a.inv_dR;
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
    a.cpa_du = a.cpa * a.inv_du;
    a.spa_du = a.spa * a.inv_du;
    a.dRA = dRA;
    a.dDec = dDec;
    a.ph_u = 256.0 * dRA;
    a.ph_v = 256.0 * dDec;
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

// Transform: the general image -> complex spectrum in XT (column stride CS);
// a swept profile -> real spectrum (column stride N/2 + 2).  Returns the
// geometry the sampler must use.
// buf2: the spectrum when the image column pass cannot run in place
// (four_step); *spec receives where the spectrum is.
template <typename T>
static int transform(const T *src, bool profile, const SweepArgs &sw, const Geom &g, void *buf,
                     hipStream_t s, Geom &gs, void *buf2 = nullptr, void **spec = nullptr) {
    FftJob<T> j{src, sw, g, (g.Q + 1) & ~1, buf, s, buf2};
    if (spec) *spec = buf;
    if (!profile && four_step<T>(g.N)) {
        if (!buf2 || !spec) return fail(GAL_ERR_SIZE, "Nxy=%d unsupported here", g.N);
        *spec = buf2;
    }
    if (profile) {
        j.g.CS = g.N / 2 + 2;
        gs = j.g;
        int rc = run_fft<T>(K_ROWS_SYM, j);
        if (rc) return rc;
        return run_fft<T>(K_COLS_SYM, j);
    }
    gs = g;
    if (four_step<T>(g.N)) gs.CS = 2 * g.P + 1;
    int rc = run_fft<T>(K_ROWS_IMG, j);
    if (rc) return rc;
    return run_fft<T>(K_COLS, j);
}

template <typename T>
static int sample(bool real_spec, const void *S, const Geom &gs, const SampleArgs &sa,
                  const Obs<T> &o, T *vis, double *chi2, const WS &w, hipStream_t s) {
    const dim3 grid((unsigned)sample_blocks(o.M)), blk(SAMPLE_NT);
    int rc;
    if (real_spec) {
        if (!chi2)
            return launch("k_sample_sym_vis", k_sample_sym<T, false>, grid, blk, s, S, gs, sa, o.u,
                          o.v, nullptr, nullptr, nullptr, vis, o.perm, w.partials, w.ctl);
        rc = launch("k_sample_sym_chi2", k_sample_sym<T, true>, grid, blk, s, S, gs, sa, o.u, o.v,
                    o.re, o.im, o.w, nullptr, nullptr, w.partials, w.ctl);
    } else {
        if (!chi2)
            return launch("k_sample_vis", k_sample<T, false>, grid, blk, s, S, gs, sa, o.u, o.v,
                          nullptr, nullptr, nullptr, vis, o.perm, w.partials, w.ctl);
        rc = launch("k_sample_chi2", k_sample<T, true>, grid, blk, s, S, gs, sa, o.u, o.v, o.re,
                    o.im, o.w, nullptr, nullptr, w.partials, w.ctl);
    }
    if (rc) return rc;
    return launch("k_reduce", k_reduce, dim3(1), dim3(REDUCE_NT), s, w.partials, (int)grid.x, chi2);
}

// Mixed-radix sizes: the image (a profile swept into the workspace first)
// through k_mr_rows and k_mr_cols into the complex spectrum layout of the
// general path, with the twiddle table of N filled at the head of the call.
template <typename T>
static int transform_mr(const T *src, bool profile, const SweepArgs &sw, const Geom &g,
                        const WS &w, hipStream_t s) {
    const int N = g.N;
    MrPlan prow, pcol;
    if (!mr_plan(N / 2, N, MR_ROWS_NT, prow) || !mr_plan(N, N, MR_COLS_NT, pcol))
        return fail(GAL_ERR_SIZE, "Nxy=%d: no mixed-radix schedule", N);
    c2<T> *W = (c2<T> *)w.mr;
    T *img = (T *)((char *)w.mr + align256((size_t)N * sizeof(c2<T>)));
    int rc = launch("k_mr_twiddles", k_mr_twiddles<T>, dim3((N + 255) / 256), dim3(256), s, W, N);
    if (rc) return rc;
    if (profile) {
        const int64_t n = (int64_t)N * N;
        rc = launch("k_sweep", k_sweep<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, src, sw,
                    N, img);
        if (rc) return rc;
        src = img;
    }
    rc = launch("k_mr_rows", k_mr_rows<T>, dim3(N), dim3(MR_ROWS_NT), s, src, g, prow,
                (const c2<T> *)W, w.xt);
    if (rc) return rc;
    return launch("k_mr_cols", k_mr_cols<T>, dim3(g.Q), dim3(MR_COLS_NT), s, g, pcol,
                  (const c2<T> *)W, w.xt);
}

template <typename T>
static int run_carved(const T *src, bool profile, const SweepArgs &sw, const Geom &g, double dxy,
                      const Obs<T> &o, double PA, double dRA, double dDec, double inc, T *vis,
                      double *chi2, const WS &w, hipStream_t s) {
    Geom gs;
    void *S = nullptr;
    bool real_spec = profile;
    int rc;
    if (w.mr) {
        rc = transform_mr<T>(src, profile, sw, g, w, s);
        gs = g;
        S = w.xt;
        real_spec = false;
    } else {
        rc = transform<T>(src, profile, sw, g, w.xt, s, gs, w.spec2, &S);
    }
    if (rc) return rc;
    const SampleArgs sa = make_sample(g, o.M, dxy, PA, dRA, dDec, inc);
    return sample<T>(real_spec, S, gs, sa, o, vis, chi2, w, s);
}

template <typename T>
static int run_path(const T *src, bool profile, const SweepArgs &sw, const Geom &g, double dxy,
                    const Obs<T> &o, double PA, double dRA, double dDec, double inc, T *vis,
                    double *chi2, void *ws, size_t ws_bytes_, hipStream_t s) {
    int rc = ensure_init();
    if (rc) return rc;
    WS w;
    rc = carve<T>(ws, ws_bytes_, g.N, o.M, w);
    if (rc) return rc;
    return run_carved<T>(src, profile, sw, g, dxy, o, PA, dRA, dDec, inc, vis, chi2, w, s);
}

// ---------------------------------------------------------------------------
// gradient path: forward transform, sample + scatter of the residuals, the
// transposed passes (adjoint.h).  Workspace: [control][partials][S][A][gI]
constexpr int GRAD_NR_MAX = 8192;  // profile bins held in LDS by the transposed sweep

template <typename T>
static size_t grad_ws_bytes(int N, int64_t M, int Nr) {
    const size_t xt = align256((size_t)(N / 2 + 1) * (size_t)(N + 2) * sizeof(c2<T>));
    return ws_bytes<T>(N, M) + xt +
           align256((size_t)GI_COPIES * (size_t)(Nr > 0 ? Nr : 1) * sizeof(double));
}

// values per thread in the adjoint FFT passes (more threads per block: a
// single job's few hundred row pairs leave the CUs short of waves)
constexpr int ADJ_E = 4;

// Row-pair groups per block of the transposed sweep, which flushes its
// histogram once per block: as many as leave about two rounds of blocks
// on the chip (3 resident per CU), at most ADJ_PPB_MAX.
constexpr int ADJ_PPB_MAX = 4;
static int adj_ppb(int groups, int jobs) {
    const int per = (int)(((int64_t)groups * jobs) / (2 * 3 * 256));
    return per < 1 ? 1 : (per > ADJ_PPB_MAX ? ADJ_PPB_MAX : per);
}

template <typename T, int N>
static int launch_adjoint(bool profile, const Geom &gs, int Qe, const SweepArgs &sw, void *A,
                          T *grad, double *gI, hipStream_t s) {
    constexpr int B = cols_B(N);
    using C = CfgE<T, N, B, ADJ_E>;
    if (profile) {
        int rc = launch("k_adj_cols_sym", k_adj_cols_sym<T, C>, dim3((Qe / 2 + B - 1) / B),
                        dim3(C::NT), s, gs, Qe, A);
        if (rc) return rc;
        const int groups = (N / 4 + 1 + B - 1) / B;
        const int ppb = adj_ppb(groups, 1);
        using CH = CfgE<T, N / 2, B, ADJ_E>;  // rows: half-length transforms of even rows
        return launch_sm("k_adj_rows_sym", k_adj_rows_sym<T, CH>, dim3((groups + ppb - 1) / ppb),
                         dim3(CH::NT), (unsigned)(sw.Nr * sizeof(double)), s, gs, A, sw, gI, ppb);
    }
    int rc = launch("k_adj_cols", k_adj_cols<T, C>, dim3((gs.Q + B - 1) / B), dim3(C::NT), s, gs,
                    A);
    if (rc) return rc;
    return launch("k_adj_rows", k_adj_rows<T, C>, dim3((N / 2 + B - 1) / B), dim3(C::NT), s, gs,
                  A, grad);
}

template <typename T>
static int dispatch_adjoint(bool profile, const Geom &gs, int Qe, const SweepArgs &sw, void *A,
                            T *grad, double *gI, hipStream_t s) {
    switch (gs.N) {
        case 16: return launch_adjoint<T, 16>(profile, gs, Qe, sw, A, grad, gI, s);
        case 32: return launch_adjoint<T, 32>(profile, gs, Qe, sw, A, grad, gI, s);
        case 64: return launch_adjoint<T, 64>(profile, gs, Qe, sw, A, grad, gI, s);
        case 128: return launch_adjoint<T, 128>(profile, gs, Qe, sw, A, grad, gI, s);
        case 256: return launch_adjoint<T, 256>(profile, gs, Qe, sw, A, grad, gI, s);
        case 512: return launch_adjoint<T, 512>(profile, gs, Qe, sw, A, grad, gI, s);
        case 1024: return launch_adjoint<T, 1024>(profile, gs, Qe, sw, A, grad, gI, s);
        case 2048: return launch_adjoint<T, 2048>(profile, gs, Qe, sw, A, grad, gI, s);
        case 4096: return launch_adjoint<T, 4096>(profile, gs, Qe, sw, A, grad, gI, s);
        case 8192: return launch_adjoint<T, 8192>(profile, gs, Qe, sw, A, grad, gI, s);
        default: return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", gs.N);
    }
}

template <typename T>
static int grad_path(const T *src, bool profile, const SweepArgs &sw, const Geom &g, double dxy,
                     const Obs<T> &o, double PA, double dRA, double dDec, double inc,
                     double *chi2, T *grad, void *ws, size_t ws_bytes_, hipStream_t s) {
    int rc = ensure_init();
    if (rc) return rc;
    if (profile && sw.Nr > GRAD_NR_MAX)
        return fail(GAL_ERR_SIZE, "profile gradient: Nr=%d above %d", sw.Nr, GRAD_NR_MAX);
    if (profile) {
        // the transposed sweep keeps Nr bins in LDS beside the FFT buffer
        const size_t lds = (size_t)cols_B(g.N) * (size_t)g.N * sizeof(c2<T>) +
                           (size_t)sw.Nr * sizeof(double);
        if (lds > (size_t)160 * 1024)
            return fail(GAL_ERR_SIZE, "profile gradient: Nr=%d too large for Nxy=%d", sw.Nr, g.N);
    }
    const int Nr = profile ? sw.Nr : 0;
    const size_t need = grad_ws_bytes<T>(g.N, o.M, Nr);
    if (!ws) return fail(GAL_ERR_NULL, "workspace is NULL");
    if (ws_bytes_ < need)
        return fail(GAL_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes_, need);
    WS w;
    rc = carve<T>(ws, ws_bytes_, g.N, o.M, w);
    if (rc) return rc;
    const size_t xt = align256((size_t)(g.N / 2 + 1) * (size_t)(g.N + 2) * sizeof(c2<T>));
    void *A = (char *)w.xt + xt;
    double *gI = (double *)((char *)A + xt);
    Geom gs;
    rc = transform<T>(src, profile, sw, g, w.xt, s, gs);
    if (rc) return rc;
    const int Qe = (g.Q + 1) & ~1;
    const int64_t a_elems = profile ? (int64_t)Qe * gs.CS : (int64_t)2 * gs.Q * gs.CS;
    // the scatter grid and, for profiles, the bin accumulator copies
    {
        const int64_t ab = a_elems * (int64_t)sizeof(T);
        const int64_t gb = profile ? (int64_t)GI_COPIES * Nr * (int64_t)sizeof(double) : 0;
        rc = launch("k_zero", k_zero16, dim3(zero_grid(ab + gb)), dim3(256), s, A, ab, (void *)gI,
                    gb);
    }
    if (rc) return rc;
    const SampleArgs sa = make_sample(g, o.M, dxy, PA, dRA, dDec, inc);
    const dim3 grid((unsigned)sample_blocks(o.M)), blk(SAMPLE_NT);
    if (profile)
        rc = launch("k_sample_scatter_sym", k_sample_scatter<T, true>, grid, blk, s, w.xt, A, gs,
                    sa, o.u, o.v, o.re, o.im, o.w, w.partials, w.ctl);
    else
        rc = launch("k_sample_scatter", k_sample_scatter<T, false>, grid, blk, s, w.xt, A, gs, sa,
                    o.u, o.v, o.re, o.im, o.w, w.partials, w.ctl);
    if (rc) return rc;
    rc = launch("k_reduce", k_reduce, dim3(1), dim3(REDUCE_NT), s, w.partials, (int)grid.x, chi2);
    if (rc) return rc;
    rc = dispatch_adjoint<T>(profile, gs, Qe, sw, A, grad, profile ? gI : nullptr, s);
    if (rc) return rc;
    if (profile)
        rc = launch("k_sum_bins", k_sum_bins<T>, dim3((Nr + 255) / 256), dim3(256), s, gI, Nr, grad);
    return rc;
}

// ---------------------------------------------------------------------------
// geometry gradient: chi^2 and d chi^2 / d (PA, dRA, dDec, inc)
template <typename T, int N>
static int rows_tangent_n(const FftJob<T> &j) {
    constexpr int B = cols_B(N);
    using C = CfgE<T, N, B, 8>;
    const int pairs = N / 4 + 1;
    return launch("k_rows_sym_dinc", k_rows_sym<T, C, true>, dim3((pairs + B - 1) / B), dim3(C::NT),
                  j.s, j.src, j.sw, j.g, j.Qe, j.buf);
}

// the real spectrum of d image / d inc of a swept profile (same passes)
template <typename T>
static int transform_tangent(const T *I, const SweepArgs &sw, const Geom &g, void *buf,
                             hipStream_t s) {
    FftJob<T> j{I, sw, g, (g.Q + 1) & ~1, buf, s};
    j.g.CS = g.N / 2 + 2;
    int rc;
    switch (g.N) {
        case 16: rc = rows_tangent_n<T, 16>(j); break;
        case 32: rc = rows_tangent_n<T, 32>(j); break;
        case 64: rc = rows_tangent_n<T, 64>(j); break;
        case 128: rc = rows_tangent_n<T, 128>(j); break;
        case 256: rc = rows_tangent_n<T, 256>(j); break;
        case 512: rc = rows_tangent_n<T, 512>(j); break;
        case 1024: rc = rows_tangent_n<T, 1024>(j); break;
        case 2048: rc = rows_tangent_n<T, 2048>(j); break;
        case 4096: rc = rows_tangent_n<T, 4096>(j); break;
        case 8192: rc = rows_tangent_n<T, 8192>(j); break;
        default: return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", g.N);
    }
    if (rc) return rc;
    return run_fft<T>(K_COLS_SYM, j);
}

// [control 256][GEO_N x partials][spectrum][tangent spectrum]
template <typename T>
static size_t geo_ws_bytes(int N, int64_t M) {
    const size_t xt = align256((size_t)(N / 2 + 1) * (size_t)(N + 2) * sizeof(c2<T>));
    return 256 + align256((size_t)GEO_N * sample_blocks(M) * sizeof(double)) + 2 * xt;
}

template <typename T>
static int geograd_path(const T *src, bool profile, const SweepArgs &sw, const Geom &g, double dxy,
                        const Obs<T> &o, double PA, double dRA, double dDec, double inc,
                        double *chi2, double *dgeo, void *ws, size_t ws_bytes_, hipStream_t s) {
    int rc = ensure_init();
    if (rc) return rc;
    if (!ws) return fail(GAL_ERR_NULL, "workspace is NULL");
    const size_t need = geo_ws_bytes<T>(g.N, o.M);
    if (ws_bytes_ < need)
        return fail(GAL_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes_, need);
    if (((uintptr_t)ws & 255) != 0) return fail(GAL_ERR_WORKSPACE, "workspace not 256-byte aligned");
    const int64_t nblk = sample_blocks(o.M);
    char *p = (char *)ws;
    Control *ctl = (Control *)p;
    double *partials = (double *)(p + 256);
    const size_t xt = align256((size_t)(g.N / 2 + 1) * (size_t)(g.N + 2) * sizeof(c2<T>));
    void *S = p + 256 + align256((size_t)GEO_N * nblk * sizeof(double));
    void *St = (char *)S + xt;
    Geom gs;
    rc = transform<T>(src, profile, sw, g, S, s, gs);
    if (rc) return rc;
    if (profile) {
        rc = transform_tangent<T>(src, sw, g, St, s);
        if (rc) return rc;
    }
    const SampleArgs sa = make_sample(g, o.M, dxy, PA, dRA, dDec, profile ? 0.0 : inc);
    const double sinc = profile ? 0.0 : std::sin(inc);
    const dim3 grid((unsigned)nblk), blk(SAMPLE_NT);
    if (profile)
        rc = launch("k_sample_geo_sym", k_sample_geo<T, true>, grid, blk, s, (const T *)S,
                    (const T *)St, gs, sa, sinc, o.u, o.v, o.re, o.im, o.w, partials, ctl);
    else
        rc = launch("k_sample_geo", k_sample_geo<T, false>, grid, blk, s, (const T *)S,
                    (const T *)nullptr, gs, sa, sinc, o.u, o.v, o.re, o.im, o.w, partials, ctl);
    if (rc) return rc;
    return launch("k_reduce_geo", k_reduce_geo, dim3(GEO_N), dim3(REDUCE_NT), s, partials,
                  (int)nblk, chi2, dgeo);
}

// ---------------------------------------------------------------------------
// autotuner: time every variant of every pass for one image size
template <typename T>
static int autotune(int N, double frac, void *stream, int *chosen_out, double *times) {
    if (!pow2_in_range(N)) return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", N);
    if (!(frac > 0.0 && frac <= 1.0)) return fail(GAL_ERR_SCALAR, "frac must be in (0, 1]");
    int rc = ensure_init();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t img_bytes = (size_t)N * N * sizeof(T);
    const size_t buf_bytes = (size_t)(N / 2 + 1) * (N + 2) * sizeof(c2<T>);
    void *img = nullptr, *buf = nullptr;
    GAL_HIP(hipMalloc(&img, img_bytes + 64));
    if (hipMalloc(&buf, buf_bytes) != hipSuccess) {
        (void)hipFree(img);
        return fail(GAL_ERR_WORKSPACE, "autotune: out of device memory");
    }
    (void)hipMemsetAsync(img, 0, img_bytes + 64, s);
    (void)hipMemsetAsync(buf, 0, buf_bytes, s);
    // a flat profile of 2 samples covering the image: every pixel inside
    T prof[2] = {T(1), T(1)};
    T *I = (T *)((char *)img + img_bytes);
    (void)hipMemcpyAsync(I, prof, sizeof(prof), hipMemcpyHostToDevice, s);
    const double dxy = 1.0;
    const SweepArgs sw = make_sweep(2, 0.0, 2.0 * N, dxy, 0.0);
    Geom g = geom_full(N);
    const int m = (int)std::floor(frac * (N / 2 - 1)) + 2;
    g.Q = min_c(g.Q, m);
    g.P = min_c(g.P, m);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const bool tm_was = g_tm_on;
    g_tm_on = false;
    int best[NKIND];
    for (int kind = 0; kind < NKIND && rc == GAL_OK; ++kind) {
        FftJob<T> j{(kind == K_ROWS_SYM) ? I : (const T *)img, sw, g, (g.Q + 1) & ~1, buf, s};
        if (kind == K_ROWS_SYM || kind == K_COLS_SYM) j.g.CS = N / 2 + 2;
        float best_ms = 1e30f;
        best[kind] = 0;
        const int nvar = N >= 256 ? NVAR : 1;
        if (times)
            for (int var = 0; var < NVAR; ++var) times[kind * NVAR + var] = -1.0;
        for (int var = 0; var < nvar && rc == GAL_OK; ++var) {
            FftFn<T> f = fft_fn<T>(N, kind, var);
            for (int it = 0; it < 3 && rc == GAL_OK; ++it) rc = f(j);
            const int reps = 20;
            (void)hipEventRecord(e0, s);
            for (int it = 0; it < reps && rc == GAL_OK; ++it) rc = f(j);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) rc = fail(GAL_ERR_HIP, "autotune sync");
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (times) times[kind * NVAR + var] = (double)ms / reps;
            if (ms < best_ms) {
                best_ms = ms;
                best[kind] = var;
            }
        }
    }
    g_tm_on = tm_was;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(img);
    (void)hipFree(buf);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int kind = 0; kind < NKIND; ++kind) {
            g_choice[sizeof(T) == 8 ? 0 : 1][log2i(N)][kind] = best[kind];
            if (chosen_out) chosen_out[kind] = best[kind];
        }
    }
    return GAL_OK;
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
    double rho_min;  // shortest baseline (image-size criterion (iia))
    void *buf;      // one allocation: u, v, re, im, w, perm (locality order)
    void *u, *v, *re, *im, *w;
    int32_t *perm;  // perm[k] = registration index of stored point k
};

// A batch plan (see batch.h): per-job descriptors, sample groups, FFT groups
// and the workspace layout.  Built on the host only; where the device table
// lives depends on the caller (own allocation or the workspace).
struct BatchPlan {
    int n = 0;
    bool grads = false;
    std::vector<JobDesc> jobs;
    std::vector<SGroup> groups;     // sorted by sample class
    std::vector<int> job_group;     // job -> group
    struct FGroup {
        int prec, kind, N, list_off, count, maxQ, maxQe, maxNr;
    };
    std::vector<FGroup> fgroups;    // FFT groups (all jobs)
    std::vector<FGroup> agroups;    // adjoint groups (gradient jobs)
    std::vector<int> lists;
    struct SClass {
        int prec;
        int kc;                     // kinds: 0 images, 1 profiles, 2 both; + 3: scenes
        int group_off, count, blocks;
        bool multi;                 // some group takes several chunks per block
    };
    std::vector<SClass> sclasses;
    size_t table_bytes = 0;         // jobs | groups | lists | job_group
    size_t zero_begin = 0, zero_end = 0;  // scatter grids and bin accumulators
    size_t ws_need = 0;
};

struct gal_batch {
    int device = 0;
    BatchPlan plan;
    void *dtab = nullptr;           // device copy of the plan's table
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
    if (!fwd_size(Nxy) || M < 0) return 0;
    return ws_bytes<double>(Nxy, M);
}
size_t gal_workspace_bytes_f(int Nxy, int64_t M) {
    if (!fwd_size(Nxy) || M < 0) return 0;
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
    int rc = check_image_scalars(Nxy, dxy, 0.0, 0.0, 0.0, inc, true);
    if (rc) return rc;
    rc = check_profile(Nr, Rmin, dR);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const SweepArgs sw = make_sweep(Nr, Rmin, dR, dxy, inc);
    const int64_t n = (int64_t)Nxy * Nxy;
    return launch("k_sweep", k_sweep<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, I, sw,
                  Nxy, image);
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
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc, true);
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
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc, true);
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
    Geom gs;
    rc = transform<T>(image, false, SweepArgs{}, g, w.xt, s, gs);
    if (rc) return rc;
    const int64_t n = (int64_t)Nxy * (Nxy / 2 + 1);
    return launch("k_spec_out", k_spec_out<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), s,
                  w.xt, g, spec);
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
    const int64_t n = (int64_t)(Nxy / 2 + 1) * (2 * g.P + 1);
    rc = launch("k_spec_in", k_spec_in<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, spec, g,
                w.xt);
    if (rc) return rc;
    const SampleArgs sa = make_sample(g, M, dxy, PA, dRA, dDec, inc);
    const Obs<T> o{u, v, nullptr, nullptr, nullptr, M, nullptr};
    return sample<T>(false, w.xt, g, sa, o, vis, nullptr, w, s);
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
// Locality order of a dataset: position along a Hilbert curve over a
// 65536^2 grid spanning [-rho_max, rho_max]^2.  Neighbouring keys are
// neighbouring points and a rotation by PA keeps neighbours together, so a
// wavefront of consecutive points gathers from a few cache lines of the
// spectrum; consecutive runs of points are connected patches of the uv plane
// (a Z-order curve jumps between distant quadrants), so a sampling block's
// stencil nodes span a compact box.
static uint64_t hilbert_key(double u, double v, double rho_max) {
    const double sc = rho_max > 0.0 ? 32767.5 / rho_max : 0.0;
    double xf = (u * sc) + 32767.5, yf = (v * sc) + 32767.5;
    xf = xf < 0.0 ? 0.0 : (xf > 65535.0 ? 65535.0 : xf);
    yf = yf < 0.0 ? 0.0 : (yf > 65535.0 ? 65535.0 : yf);
    uint32_t x = (uint32_t)xf, y = (uint32_t)yf;
    constexpr uint32_t n = 65536;
    uint64_t d = 0;
    for (uint32_t s = n / 2; s > 0; s /= 2) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * s * ((3u * rx) ^ ry);
        if (ry == 0) {  // rotate the quadrant so that the sub-curve starts at its corner
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

template <typename T>
static int dataset_create(const T *u, const T *v, const T *re, const T *im, const T *w, int64_t M,
                          void *stream, gal_dataset **out) {
    if (!out) return fail(GAL_ERR_NULL, "NULL out");
    *out = nullptr;
    if (M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    if (M > (int64_t)0x7fffffff) return fail(GAL_ERR_SIZE, "M above 2^31 - 1");
    if (M > 0 && (!u || !v)) return fail(GAL_ERR_NULL, "NULL u or v");
    // an empty dataset holds (no) observations whatever the pointers are: its
    // chi^2 is 0 (empty arrays may come with NULL pointers)
    const bool has_obs = (re && im && w) || M == 0;
    if (M > 0 && (re || im || w) && !has_obs) return fail(GAL_ERR_NULL, "re, im, w: give all or none");
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
    double r2max = 0.0, r2min = M > 0 ? INFINITY : 0.0;
    for (int64_t k = 0; k < M; ++k) {
        const double uu = h[0][k], vv = h[1][k];
        const double r2 = uu * uu + vv * vv;
        if (!std::isfinite(r2)) return fail(GAL_ERR_SCALAR, "non-finite uv coordinate at %lld",
                                            (long long)k);
        r2max = r2 > r2max ? r2 : r2max;
        r2min = r2 < r2min ? r2 : r2min;
    }
    const double rho_max = std::sqrt(r2max);
    // locality order
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)M);
    for (int64_t k = 0; k < M; ++k)
        key[k] = {hilbert_key((double)h[0][k], (double)h[1][k], rho_max), (int32_t)k};
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, int32_t> &a, const std::pair<uint64_t, int32_t> &b) {
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
    ds->rho_min = std::sqrt(r2min);
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

// ---- image size (Sec. 3.4 criteria) ---------------------------------------
// smooth: N the smallest even 2^a 3^b 5^c instead of the smallest power of two
static int image_size(double rho_min, double rho_max, double f_min, double f_max, double PB,
                      double Gamma, bool smooth, int *Nxy, double *dxy) {
    if (!Nxy || !dxy) return fail(GAL_ERR_NULL, "NULL output");
    if (!(f_max > 2.0) || !std::isfinite(f_max)) return fail(GAL_ERR_SCALAR, "f_max must be > 2");
    if (!(PB >= 0.0) || !std::isfinite(PB)) return fail(GAL_ERR_SCALAR, "PB must be >= 0");
    if (!(rho_max > 0.0) || !std::isfinite(rho_max) || !(rho_min <= rho_max))
        return fail(GAL_ERR_SCALAR, "uv range [%g, %g] unusable", rho_min, rho_max);
    double du;
    if (PB > 0.0) {
        du = 1.0 / PB;  // (iib): the image spans the primary beam
    } else {
        if (!(f_min > 1.0) || !std::isfinite(f_min)) return fail(GAL_ERR_SCALAR, "f_min must be > 1");
        if (!(Gamma > 0.0) || !std::isfinite(Gamma)) return fail(GAL_ERR_SCALAR, "Gamma must be > 0");
        if (!(rho_min > 0.0)) return fail(GAL_ERR_SCALAR, "criterion (iia) needs rho_min > 0");
        du = rho_min / (Gamma * f_min);  // (iia): f_min times the largest recoverable scale
    }
    // (i): the grid reaches f_max times the longest baseline; N a power of two
    int64_t n = 2;
    while ((double)n * du / 2.0 < f_max * rho_max) {
        n *= 2;
        if (n > ((int64_t)1 << 30)) return fail(GAL_ERR_SIZE, "image size above 2^30");
    }
    if (smooth) {
        // the smallest even 2^a 3^b 5^c meeting (i): between n / 2 and n
        for (int64_t m = n / 2 + (n / 2) % 2; m <= n; m += 2) {
            if ((double)m * du / 2.0 < f_max * rho_max) continue;
            int64_t r = m;
            for (int f : {2, 3, 5})
                while (r % f == 0) r /= f;
            if (r == 1) {
                n = m;
                break;
            }
        }
    }
    *Nxy = (int)n;
    *dxy = 1.0 / ((double)n * du);
    return GAL_OK;
}
int gal_image_size(double rho_min, double rho_max, double f_min, double f_max, double PB,
                   double Gamma, int *Nxy, double *dxy) {
    return image_size(rho_min, rho_max, f_min, f_max, PB, Gamma, false, Nxy, dxy);
}
int gal_image_size_smooth(double rho_min, double rho_max, double f_min, double f_max, double PB,
                          double Gamma, int *Nxy, double *dxy) {
    return image_size(rho_min, rho_max, f_min, f_max, PB, Gamma, true, Nxy, dxy);
}

template <typename T>
static int uv_range(const T *u, const T *v, int64_t M, double *rho_min, double *rho_max) {
    if (!rho_min || !rho_max) return fail(GAL_ERR_NULL, "NULL output");
    if (M < 1) return fail(GAL_ERR_SIZE, "M < 1");
    if (!u || !v) return fail(GAL_ERR_NULL, "NULL u or v");
    double lo = INFINITY, hi = 0.0;
    for (int64_t k = 0; k < M; ++k) {
        const double uu = u[k], vv = v[k];
        const double r = std::sqrt(uu * uu + vv * vv);
        if (!std::isfinite(r)) return fail(GAL_ERR_SCALAR, "non-finite uv coordinate at %lld", (long long)k);
        lo = r < lo ? r : lo;
        hi = r > hi ? r : hi;
    }
    *rho_min = lo;
    *rho_max = hi;
    return GAL_OK;
}
int gal_uv_range_d(const double *u, const double *v, int64_t M, double *rho_min, double *rho_max) {
    return uv_range(u, v, M, rho_min, rho_max);
}
int gal_uv_range_f(const float *u, const float *v, int64_t M, double *rho_min, double *rho_max) {
    return uv_range(u, v, M, rho_min, rho_max);
}

int gal_dataset_image_size(const gal_dataset *ds, double f_min, double f_max, double PB,
                           double Gamma, int *Nxy, double *dxy) {
    if (!ds) return fail(GAL_ERR_NULL, "NULL dataset");
    if (ds->M < 1) return fail(GAL_ERR_SIZE, "empty dataset");
    return gal_image_size(ds->rho_min, ds->rho_max, f_min, f_max, PB, Gamma, Nxy, dxy);
}
int gal_dataset_image_size_smooth(const gal_dataset *ds, double f_min, double f_max, double PB,
                                  double Gamma, int *Nxy, double *dxy) {
    if (!ds) return fail(GAL_ERR_NULL, "NULL dataset");
    if (ds->M < 1) return fail(GAL_ERR_SIZE, "empty dataset");
    return gal_image_size_smooth(ds->rho_min, ds->rho_max, f_min, f_max, PB, Gamma, Nxy, dxy);
}

int gal_dataset_geometry(const gal_dataset *ds, int Nxy, double dxy, int *Q, int *P) {
    if (!ds || !Q || !P) return fail(GAL_ERR_NULL, "NULL argument");
    int rc = check_image_scalars(Nxy, dxy, 0.0, 0.0, 0.0, 0.0, true);
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
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc, true);
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
int gal_chi2Profile_ds_scratch_d(const gal_dataset *ds, const double *I, int Nr, double Rmin,
                                 double dR, int Nxy, double dxy, double inc, double PA,
                                 double dRA, double dDec, double *chi2, void *stream) {
    if (!chi2 || !ds) return fail(GAL_ERR_NULL, "NULL argument");
    if (!pow2_in_range(Nxy)) return fail(GAL_ERR_SIZE, "Nxy=%d: need a power of two in [16, 8192]", Nxy);
    const size_t need = ws_bytes<double>(Nxy, ds->M);
    if (need > (size_t)GAL_SCRATCH_BYTES)
        return fail(GAL_ERR_WORKSPACE,
                    "Nxy=%d, M=%lld needs %zu bytes of workspace; the scratch holds %zu "
                    "(use gal_chi2Profile_ds_d with a caller's workspace)",
                    Nxy, (long long)ds->M, need, (size_t)GAL_SCRATCH_BYTES);
    int rc = ensure_init();
    if (rc) return rc;
    int dev = 0;
    GAL_HIP(hipGetDevice(&dev));
    void *sp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_init_mu);
        if ((int)g_scratch_ptr.size() > dev) sp = g_scratch_ptr[dev];
    }
    if (!sp) return fail(GAL_ERR_HIP, "scratch workspace of device %d has no address", dev);
    return ds_call<double>(ds, I, true, Nr, Rmin, dR, Nxy, dxy, inc, PA, dRA, dDec, nullptr, chi2,
                           sp, (size_t)GAL_SCRATCH_BYTES, stream);
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

// ---- gradients ------------------------------------------------------------
size_t gal_grad_workspace_bytes_d(int Nxy, int64_t M, int Nr) {
    if (!pow2_in_range(Nxy) || M < 0 || Nr < 0) return 0;
    return grad_ws_bytes<double>(Nxy, M, Nr);
}
size_t gal_grad_workspace_bytes_f(int Nxy, int64_t M, int Nr) {
    if (!pow2_in_range(Nxy) || M < 0 || Nr < 0) return 0;
    return grad_ws_bytes<float>(Nxy, M, Nr);
}

template <typename T>
static int image_grad_call(const T *image, int Nxy, double dxy, const Obs<T> &o, double PA,
                           double dRA, double dDec, double inc, double *chi2, T *grad, void *ws,
                           size_t ws_bytes_, void *stream, const Geom *gpruned) {
    if (!image || !chi2 || !grad) return fail(GAL_ERR_NULL, "NULL array");
    if (o.M > 0 && (!o.u || !o.v || !o.re || !o.im || !o.w))
        return fail(GAL_ERR_NULL, "NULL observation array");
    if (o.M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);
    if (rc) return rc;
    const Geom g = gpruned ? *gpruned : geom_full(Nxy);
    return grad_path<T>(image, false, SweepArgs{}, g, dxy, o, PA, dRA, dDec, inc, chi2, grad, ws,
                        ws_bytes_, (hipStream_t)stream);
}

template <typename T>
static int profile_grad_call(const T *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                             const Obs<T> &o, double inc, double PA, double dRA, double dDec,
                             double *chi2, T *grad, void *ws, size_t ws_bytes_, void *stream,
                             const Geom *gpruned) {
    if (!I || !chi2 || !grad) return fail(GAL_ERR_NULL, "NULL array");
    if (o.M > 0 && (!o.u || !o.v || !o.re || !o.im || !o.w))
        return fail(GAL_ERR_NULL, "NULL observation array");
    if (o.M < 0) return fail(GAL_ERR_SIZE, "M < 0");
    int rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);
    if (rc) return rc;
    rc = check_profile(Nr, Rmin, dR);
    if (rc) return rc;
    const Geom g = gpruned ? *gpruned : geom_full(Nxy);
    return grad_path<T>(I, true, make_sweep(Nr, Rmin, dR, dxy, inc), g, dxy, o, PA, dRA, dDec, 0.0,
                        chi2, grad, ws, ws_bytes_, (hipStream_t)stream);
}

#define GAL_IMAGE_GRAD(SFX, T)                                                                  \
    int gal_chi2Image_grad_##SFX(const T *image, int Nxy, double dxy, const T *u, const T *v,   \
                                 const T *re, const T *im, const T *w, int64_t M, double PA,    \
                                 double dRA, double dDec, double inc, double *chi2, T *grad,    \
                                 void *ws, size_t ws_bytes_, void *stream) {                    \
        return image_grad_call<T>(image, Nxy, dxy, Obs<T>{u, v, re, im, w, M, nullptr}, PA, dRA, \
                                  dDec, inc, chi2, grad, ws, ws_bytes_, stream, nullptr);       \
    }
GAL_IMAGE_GRAD(d, double)
GAL_IMAGE_GRAD(f, float)

#define GAL_PROFILE_GRAD(SFX, T)                                                                \
    int gal_chi2Profile_grad_##SFX(const T *I, int Nr, double Rmin, double dR, int Nxy,         \
                                   double dxy, const T *u, const T *v, const T *re,             \
                                   const T *im, const T *w, int64_t M, double inc, double PA,   \
                                   double dRA, double dDec, double *chi2, T *grad, void *ws,    \
                                   size_t ws_bytes_, void *stream) {                            \
        return profile_grad_call<T>(I, Nr, Rmin, dR, Nxy, dxy,                                  \
                                    Obs<T>{u, v, re, im, w, M, nullptr}, inc, PA, dRA, dDec,    \
                                    chi2, grad, ws, ws_bytes_, stream, nullptr);                \
    }
GAL_PROFILE_GRAD(d, double)
GAL_PROFILE_GRAD(f, float)

template <typename T>
static int ds_grad(const gal_dataset *ds, int Nxy, double dxy, Geom &g, Obs<T> &o) {
    if (!ds) return fail(GAL_ERR_NULL, "NULL dataset");
    if (ds->precision != (int)sizeof(T))
        return fail(GAL_ERR_UNSUPPORTED, "dataset precision %d differs from the call", ds->precision);
    if (!ds->re) return fail(GAL_ERR_UNSUPPORTED, "dataset holds no observations");
    if (!pow2_in_range(Nxy)) return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", Nxy);
    if (!(dxy >= DXY_MIN) || !std::isfinite(dxy)) return fail(GAL_ERR_SCALAR, "dxy must be >= 1e-100");
    const double du = 1.0 / ((double)Nxy * dxy);
    if (!(ds->rho_max < ((double)(Nxy / 2) - 1.0) * du))
        return fail(GAL_ERR_UV_RANGE, "rho_max = %.6g lambda reaches beyond the half spectrum",
                    ds->rho_max);
    g = geom_pruned(Nxy, dxy, ds->rho_max);
    o = Obs<T>{(const T *)ds->u, (const T *)ds->v, (const T *)ds->re, (const T *)ds->im,
               (const T *)ds->w, ds->M, nullptr};
    return GAL_OK;
}

#define GAL_IMAGE_GRAD_DS(SFX, T)                                                               \
    int gal_chi2Image_grad_ds_##SFX(const gal_dataset *ds, const T *image, int Nxy, double dxy, \
                                    double PA, double dRA, double dDec, double inc,             \
                                    double *chi2, T *grad, void *ws, size_t ws_bytes_,          \
                                    void *stream) {                                             \
        Geom g;                                                                                 \
        Obs<T> o;                                                                               \
        int rc = ds_grad<T>(ds, Nxy, dxy, g, o);                                                \
        if (rc) return rc;                                                                      \
        return image_grad_call<T>(image, Nxy, dxy, o, PA, dRA, dDec, inc, chi2, grad, ws,       \
                                  ws_bytes_, stream, &g);                                       \
    }
GAL_IMAGE_GRAD_DS(d, double)
GAL_IMAGE_GRAD_DS(f, float)

#define GAL_PROFILE_GRAD_DS(SFX, T)                                                             \
    int gal_chi2Profile_grad_ds_##SFX(const gal_dataset *ds, const T *I, int Nr, double Rmin,   \
                                      double dR, int Nxy, double dxy, double inc, double PA,    \
                                      double dRA, double dDec, double *chi2, T *grad, void *ws, \
                                      size_t ws_bytes_, void *stream) {                         \
        Geom g;                                                                                 \
        Obs<T> o;                                                                               \
        int rc = ds_grad<T>(ds, Nxy, dxy, g, o);                                                \
        if (rc) return rc;                                                                      \
        return profile_grad_call<T>(I, Nr, Rmin, dR, Nxy, dxy, o, inc, PA, dRA, dDec, chi2,     \
                                    grad, ws, ws_bytes_, stream, &g);                           \
    }
GAL_PROFILE_GRAD_DS(d, double)
GAL_PROFILE_GRAD_DS(f, float)

size_t gal_geograd_workspace_bytes_d(int Nxy, int64_t M) {
    if (!pow2_in_range(Nxy) || M < 0) return 0;
    return geo_ws_bytes<double>(Nxy, M);
}
size_t gal_geograd_workspace_bytes_f(int Nxy, int64_t M) {
    if (!pow2_in_range(Nxy) || M < 0) return 0;
    return geo_ws_bytes<float>(Nxy, M);
}

#define GAL_IMAGE_GEOGRAD_DS(SFX, T)                                                            \
    int gal_chi2Image_geograd_ds_##SFX(const gal_dataset *ds, const T *image, int Nxy,          \
                                       double dxy, double PA, double dRA, double dDec,          \
                                       double inc, double *chi2, double *dgeo, void *ws,        \
                                       size_t ws_bytes_, void *stream) {                        \
        Geom g;                                                                                 \
        Obs<T> o;                                                                               \
        int rc = ds_grad<T>(ds, Nxy, dxy, g, o);                                                \
        if (rc) return rc;                                                                      \
        if (!image || !chi2 || !dgeo) return fail(GAL_ERR_NULL, "NULL array");                  \
        rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);                                 \
        if (rc) return rc;                                                                      \
        return geograd_path<T>(image, false, SweepArgs{}, g, dxy, o, PA, dRA, dDec, inc, chi2,  \
                               dgeo, ws, ws_bytes_, (hipStream_t)stream);                       \
    }
GAL_IMAGE_GEOGRAD_DS(d, double)
GAL_IMAGE_GEOGRAD_DS(f, float)

#define GAL_PROFILE_GEOGRAD_DS(SFX, T)                                                          \
    int gal_chi2Profile_geograd_ds_##SFX(const gal_dataset *ds, const T *I, int Nr,             \
                                         double Rmin, double dR, int Nxy, double dxy,           \
                                         double inc, double PA, double dRA, double dDec,        \
                                         double *chi2, double *dgeo, void *ws,                  \
                                         size_t ws_bytes_, void *stream) {                      \
        Geom g;                                                                                 \
        Obs<T> o;                                                                               \
        int rc = ds_grad<T>(ds, Nxy, dxy, g, o);                                                \
        if (rc) return rc;                                                                      \
        if (!I || !chi2 || !dgeo) return fail(GAL_ERR_NULL, "NULL array");                      \
        rc = check_image_scalars(Nxy, dxy, PA, dRA, dDec, inc);                                 \
        if (rc) return rc;                                                                      \
        rc = check_profile(Nr, Rmin, dR);                                                       \
        if (rc) return rc;                                                                      \
        return geograd_path<T>(I, true, make_sweep(Nr, Rmin, dR, dxy, inc), g, dxy, o, PA, dRA, \
                               dDec, inc, chi2, dgeo, ws, ws_bytes_, (hipStream_t)stream);      \
    }
GAL_PROFILE_GEOGRAD_DS(d, double)
GAL_PROFILE_GEOGRAD_DS(f, float)

// ---- batches --------------------------------------------------------------
// Plan a job list: checks, geometry, scenes (jobs whose visibilities add up),
// sample groups (scenes on the same dataset with the same member kinds and
// grids, <= KMAX jobs unless one scene is larger), FFT groups (same
// precision, kind and size; jobs that read another's spectrum have none),
// adjoint groups (gradient jobs that own a spectrum), workspace layout
// starting at `base`: [partials][spectra][scatter grids][bin accumulators].
static int plan_batch(const gal_job *jobs, int n, void *const *grads, size_t base,
                      BatchPlan &P) {
    if (n < 1) return fail(GAL_ERR_SIZE, "a batch needs at least one job");
    if (!jobs) return fail(GAL_ERR_NULL, "NULL jobs");
    int dev = 0;
    GAL_HIP(hipGetDevice(&dev));
    P = BatchPlan();
    P.n = n;
    P.jobs.resize(n);
    P.job_group.assign(n, -1);
    for (int i = 0; i < n; ++i) {
        const gal_job &J = jobs[i];
        void *gr = grads ? grads[i] : nullptr;
        if (J.scene < 0 || J.share < 0 || J.share > n)
            return fail(GAL_ERR_UNSUPPORTED, "job %d: scene and share must be >= 0, share <= n", i);
        if (!J.ds || !J.geo || (!J.model && !J.share))
            return fail(GAL_ERR_NULL, "job %d: NULL dataset, model or geo", i);
        if (!J.ds->re && gr) return fail(GAL_ERR_UNSUPPORTED, "job %d: a gradient needs observations", i);
        if (J.kind != 0 && J.kind != 1) return fail(GAL_ERR_UNSUPPORTED, "job %d: kind must be 0 or 1", i);
        if (!pow2_in_range(J.Nxy)) return fail(GAL_ERR_SIZE, "job %d: Nxy unsupported", i);
        if (!(J.dxy >= DXY_MIN) || !std::isfinite(J.dxy)) return fail(GAL_ERR_SCALAR, "job %d: dxy must be >= 1e-100", i);
        if (J.ds->device != dev) return fail(GAL_ERR_UNSUPPORTED, "job %d: dataset on another device", i);
        const double du = 1.0 / ((double)J.Nxy * J.dxy);
        if (!(J.ds->rho_max < ((double)(J.Nxy / 2) - 1.0) * du))
            return fail(GAL_ERR_UV_RANGE, "job %d: dataset rho_max reaches beyond the half spectrum", i);
        if (J.share) {
            const int o = J.share - 1;
            const gal_job &O = jobs[o];
            if (o == i || O.share) return fail(GAL_ERR_UNSUPPORTED, "job %d: shares the spectrum of a job that shares one", i);
            if (!J.scene || O.scene != J.scene)
                return fail(GAL_ERR_UNSUPPORTED, "job %d: shares a spectrum outside its scene", i);
            if (O.kind != J.kind || O.Nxy != J.Nxy || O.dxy != J.dxy || O.ds != J.ds)
                return fail(GAL_ERR_UNSUPPORTED, "job %d: shares a spectrum of another kind or grid", i);
            if (gr) return fail(GAL_ERR_UNSUPPORTED, "job %d: a sharing job's gradient goes to the owner's output", i);
            continue;  // described below, from its owner
        }
        if (J.kind == 1 && J.Nr < 2) return fail(GAL_ERR_SIZE, "job %d: Nr < 2", i);
        if (gr && J.kind == 1) {
            if (J.Nr > GRAD_NR_MAX) return fail(GAL_ERR_SIZE, "job %d: gradient needs Nr <= %d", i, GRAD_NR_MAX);
            const size_t lds = (size_t)cols_B(J.Nxy) * J.Nxy * 2 * (size_t)J.ds->precision +
                               (size_t)J.Nr * sizeof(double);
            if (lds > (size_t)160 * 1024) return fail(GAL_ERR_SIZE, "job %d: Nr too large for Nxy", i);
        }
        const Geom g = geom_pruned(J.Nxy, J.dxy, J.ds->rho_max);
        JobDesc &d = P.jobs[i];
        d = JobDesc{};
        d.src = J.model;
        d.geo = J.geo;
        d.grad = gr;
        d.vis = J.vis;
        d.kind = J.kind;
        d.N = J.Nxy;
        d.Nr = J.kind == 1 ? J.Nr : 0;
        d.Q = g.Q;
        d.P = g.P;
        d.Qe = (g.Q + 1) & ~1;
        d.CS = J.kind == 1 ? J.Nxy / 2 + 2 : g.CS;
        d.dxy = J.dxy;
        P.grads = P.grads || gr;
    }
    // scenes: units of the sampling pass (a job with scene 0 is alone)
    std::vector<std::vector<int>> units;
    {
        std::vector<std::pair<int, int>> first;  // scene id -> unit
        for (int i = 0; i < n; ++i) {
            const int sid = jobs[i].scene;
            int u = -1;
            if (sid) {
                for (const auto &f : first)
                    if (f.first == sid) u = f.second;
            }
            if (u < 0) {
                u = (int)units.size();
                units.emplace_back();
                if (sid) first.push_back({sid, u});
            } else if (jobs[units[u][0]].ds != jobs[i].ds) {
                return fail(GAL_ERR_UNSUPPORTED, "job %d: a scene spans two datasets", i);
            }
            units[u].push_back(i);
        }
    }
    // a unit's member kinds and grids; units with equal signatures on one
    // dataset share a group
    auto same_sig = [&](const std::vector<int> &a, const std::vector<int> &c) {
        if (a.size() != c.size() || jobs[a[0]].ds != jobs[c[0]].ds) return false;
        for (size_t m = 0; m < a.size(); ++m) {
            const gal_job &x = jobs[a[m]], &y = jobs[c[m]];
            if (x.kind != y.kind || x.Nxy != y.Nxy || x.dxy != y.dxy || !x.share != !y.share ||
                !x.vis != !y.vis)
                return false;
        }
        return true;
    };
    auto kind_class = [&](const std::vector<int> &u) {
        int has = 0;
        for (int i : u) has |= jobs[i].kind == 1 ? 2 : 1;
        return has == 1 ? 0 : has == 2 ? 1 : 2;
    };
    struct GroupDraft {
        std::vector<int> units;
        int nj = 0;
    };
    std::vector<GroupDraft> drafts;
    {
        std::vector<char> used(units.size(), 0);
        for (size_t a0 = 0; a0 < units.size(); ++a0) {
            if (used[a0]) continue;
            GroupDraft G;
            for (size_t c = a0; c < units.size(); ++c) {
                if (used[c] || !same_sig(units[a0], units[c])) continue;
                if (G.nj > 0 && G.nj + (int)units[c].size() > KMAX) continue;
                used[c] = 1;
                G.units.push_back((int)c);
                G.nj += (int)units[c].size();
            }
            drafts.push_back(G);
        }
    }
    // class: precision, member kinds, and whether the scene kernel is needed
    // (several sources, a visibility output or no observations)
    auto needs_scene = [&](const std::vector<int> &u) {
        bool r = u.size() > 1 || !jobs[u[0]].ds->re;
        for (int i : u) r = r || jobs[i].vis;
        return r;
    };
    auto cls = [&](const GroupDraft &G) {
        const std::vector<int> &u = units[G.units[0]];
        return (jobs[u[0]].ds->precision == 8 ? 0 : 6) + (needs_scene(u) ? 3 : 0) + kind_class(u);
    };
    std::vector<int> order(drafts.size());
    for (size_t g = 0; g < order.size(); ++g) order[g] = (int)g;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return cls(drafts[a]) < cls(drafts[c]); });
    for (int gi : order) {
        const GroupDraft &D = drafts[gi];
        const gal_dataset *ds = jobs[units[D.units[0]][0]].ds;
        SGroup G{};
        G.u = ds->u;
        G.v = ds->v;
        G.re = ds->re;
        G.im = ds->im;
        G.w = ds->w;
        G.perm = ds->perm;
        G.M = ds->M;
        G.nchunk = (int)sample_blocks(G.M);
        G.job_off = (int)P.lists.size();
        G.nj = D.nj;
        // plain groups of few jobs take several chunks per block (one chunk
        // of one job is too little work to cover a block's set-up and memory
        // latency); scene groups and gradient runs one
        const bool scene = cls(D) % 6 >= 3;
        G.cpb = (P.grads || scene) ? 1 : (G.nj <= 2 ? 4 : (G.nj <= 4 ? 2 : 1));
        G.nblk = (G.nchunk + G.cpb - 1) / G.cpb;
        for (int u : D.units)
            for (int i : units[u]) {
                P.job_group[i] = (int)P.groups.size();
                P.lists.push_back(i);
            }
        G.sc_off = (int)P.lists.size();
        G.nsc = (int)D.units.size();
        int m = 0;
        for (int u : D.units) {
            P.lists.push_back(m);
            m += (int)units[u].size();
        }
        P.lists.push_back(m);
        const int c = cls(D);
        const int prec = c < 6 ? 8 : 4;
        const int kc = c % 6;
        if (P.sclasses.empty() || P.sclasses.back().prec != prec || P.sclasses.back().kc != kc)
            P.sclasses.push_back({prec, kc, (int)P.groups.size(), 0, 0, false});
        BatchPlan::SClass &sc = P.sclasses.back();
        G.blk0 = sc.blocks;
        sc.blocks += G.nblk;
        sc.count += 1;
        sc.multi = sc.multi || G.cpb > 1;
        P.groups.push_back(G);
    }
    auto make_groups = [&](bool grad_only, std::vector<BatchPlan::FGroup> &out) {
        std::vector<char> used(n, 0);
        for (int i = 0; i < n; ++i) {
            if (used[i] || jobs[i].share || (grad_only && !P.jobs[i].grad)) continue;
            const int prec = jobs[i].ds->precision;
            BatchPlan::FGroup f{prec, jobs[i].kind, jobs[i].Nxy, (int)P.lists.size(), 0, 0, 0, 0};
            for (int k = i; k < n; ++k) {
                if (used[k] || jobs[k].share || (grad_only && !P.jobs[k].grad)) continue;
                if (jobs[k].ds->precision != prec || jobs[k].kind != f.kind || jobs[k].Nxy != f.N)
                    continue;
                used[k] = 1;
                P.lists.push_back(k);
                f.count += 1;
                f.maxQ = max_c(f.maxQ, P.jobs[k].Q);
                f.maxQe = max_c(f.maxQe, P.jobs[k].Qe);
                f.maxNr = max_c(f.maxNr, P.jobs[k].Nr);
            }
            out.push_back(f);
        }
    };
    make_groups(false, P.fgroups);
    make_groups(true, P.agroups);
    // layout: partials per scene (at its first member), spectra, scatter
    // grids and bin accumulators per owning job
    P.table_bytes = align256(sizeof(JobDesc) * n) + align256(sizeof(SGroup) * P.groups.size()) +
                    align256(sizeof(int) * P.lists.size()) + align256(sizeof(int) * n);
    size_t off = base;
    for (const auto &u : units) {
        P.jobs[u[0]].part_off = off;
        off += align256((size_t)P.groups[P.job_group[u[0]]].nchunk * WAVES * sizeof(double));
        for (int i : u) P.jobs[i].part_off = P.jobs[u[0]].part_off;
    }
    auto spec_bytes = [&](int i) {
        const JobDesc &d = P.jobs[i];
        const size_t el = (size_t)jobs[i].ds->precision;
        return d.kind == 1 ? (size_t)d.Qe * d.CS * el : (size_t)d.Q * d.CS * 2 * el;
    };
    for (int i = 0; i < n; ++i) {
        if (jobs[i].share) continue;
        P.jobs[i].spec_off = off;
        off += align256(spec_bytes(i));
    }
    P.zero_begin = off;
    for (int i = 0; i < n; ++i) {
        if (!P.jobs[i].grad || jobs[i].share) continue;
        P.jobs[i].a_off = off;
        off += align256(spec_bytes(i));
        if (P.jobs[i].kind == 1) {
            P.jobs[i].gi_off = off;
            off += align256((size_t)GI_COPIES * P.jobs[i].Nr * sizeof(double));
        }
    }
    P.zero_end = off;
    P.ws_need = off;
    // a sharing job: the owner's transform, spectrum and gradient buffers;
    // its own geometry, scene partials and visibility output
    for (int i = 0; i < n; ++i) {
        if (!jobs[i].share) continue;
        JobDesc d = P.jobs[jobs[i].share - 1];
        d.shared = 1;
        d.geo = jobs[i].geo;
        d.vis = jobs[i].vis;
        d.part_off = P.jobs[i].part_off;
        P.jobs[i] = d;
    }
    return GAL_OK;
}

struct BatchTables {
    JobDesc *jobs;
    SGroup *groups;
    int *lists;
    int *job_group;
};

static BatchTables tables_at(const BatchPlan &P, void *base) {
    char *p = (char *)base;
    BatchTables t;
    t.jobs = (JobDesc *)p;
    p += align256(sizeof(JobDesc) * P.n);
    t.groups = (SGroup *)p;
    p += align256(sizeof(SGroup) * P.groups.size());
    t.lists = (int *)p;
    p += align256(sizeof(int) * P.lists.size());
    t.job_group = (int *)p;
    return t;
}

// host copy of the table, laid out as on the device
static std::vector<char> table_image(const BatchPlan &P) {
    std::vector<char> h(P.table_bytes, 0);
    BatchTables t = tables_at(P, h.data());
    std::memcpy(t.jobs, P.jobs.data(), sizeof(JobDesc) * P.n);
    std::memcpy(t.groups, P.groups.data(), sizeof(SGroup) * P.groups.size());
    if (!P.lists.empty()) std::memcpy(t.lists, P.lists.data(), sizeof(int) * P.lists.size());
    std::memcpy(t.job_group, P.job_group.data(), sizeof(int) * P.n);
    return h;
}

template <typename T>
static int batch_fft(const BatchPlan::FGroup &f, const BatchTables &t, char *ws, hipStream_t s) {
    FftJobB j{t.jobs, t.lists + f.list_off, f.count, f.maxQ, f.maxQe, ws, s};
    const int k1 = f.kind == 1 ? K_ROWS_SYM : K_ROWS_IMG;
    const int k2 = f.kind == 1 ? K_COLS_SYM : K_COLS;
    FftFnB r = fft_fn_b<T>(f.N, k1, chosen_var<T>(f.N, k1));
    FftFnB c = fft_fn_b<T>(f.N, k2, chosen_var<T>(f.N, k2));
    if (!r || !c) return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", f.N);
    int rc = r(j);
    if (rc) return rc;
    return c(j);
}

template <typename T, int N>
static int batch_adj_n(const BatchPlan::FGroup &f, const BatchTables &t, char *ws, hipStream_t s) {
    constexpr int B = cols_B(N);
    using C = CfgE<T, N, B, ADJ_E>;
    const int *list = t.lists + f.list_off;
    int rc;
    if (f.kind == 1) {
        rc = launch("kb_adj_cols_sym", kb_adj_cols_sym<T, C>, dim3((f.maxQe / 2 + B - 1) / B, f.count),
                    dim3(C::NT), s, t.jobs, list, ws);
        if (rc) return rc;
        using CH = CfgE<T, N / 2, B, ADJ_E>;  // rows: half-length transforms of even rows
        const int groups = (N / 4 + 1 + B - 1) / B;
        const int ppb = adj_ppb(groups, f.count);
        rc = launch_sm("kb_adj_rows_sym", kb_adj_rows_sym<T, CH>,
                       dim3((groups + ppb - 1) / ppb, f.count), dim3(CH::NT),
                       (unsigned)(f.maxNr * sizeof(double)), s, t.jobs, list, ws, ppb);
        if (rc) return rc;
        return launch("kb_grad_out", kb_grad_out<T>, dim3((f.maxNr + 255) / 256, f.count), dim3(256),
                      s, t.jobs, list, ws);
    }
    rc = launch("kb_adj_cols", kb_adj_cols<T, C>, dim3((f.maxQ + B - 1) / B, f.count), dim3(C::NT),
                s, t.jobs, list, ws);
    if (rc) return rc;
    return launch("kb_adj_rows", kb_adj_rows<T, C>, dim3((N / 2 + B - 1) / B, f.count), dim3(C::NT),
                  s, t.jobs, list, ws);
}

template <typename T>
static int batch_adj(const BatchPlan::FGroup &f, const BatchTables &t, char *ws, hipStream_t s) {
    switch (f.N) {
        case 16: return batch_adj_n<T, 16>(f, t, ws, s);
        case 32: return batch_adj_n<T, 32>(f, t, ws, s);
        case 64: return batch_adj_n<T, 64>(f, t, ws, s);
        case 128: return batch_adj_n<T, 128>(f, t, ws, s);
        case 256: return batch_adj_n<T, 256>(f, t, ws, s);
        case 512: return batch_adj_n<T, 512>(f, t, ws, s);
        case 1024: return batch_adj_n<T, 1024>(f, t, ws, s);
        case 2048: return batch_adj_n<T, 2048>(f, t, ws, s);
        case 4096: return batch_adj_n<T, 4096>(f, t, ws, s);
        case 8192: return batch_adj_n<T, 8192>(f, t, ws, s);
        default: return fail(GAL_ERR_SIZE, "Nxy=%d unsupported", f.N);
    }
}

template <typename T, int KC>
static int batch_sample(const BatchPlan::SClass &c, bool grads, const BatchTables &t, char *ws,
                        hipStream_t s) {
    const SGroup *g = t.groups + c.group_off;
    const dim3 grid(c.blocks), blk(SAMPLE_NT);
    if (KC >= 3) {  // scenes
        constexpr int K = KC >= 3 ? KC - 3 : 0;
        if (grads)
            return launch("kb_sample_scene", kb_sample_scene<T, K, true>, grid, blk, s, t.jobs, g,
                          t.lists, c.count, ws);
        return launch("kb_sample_scene", kb_sample_scene<T, K, false>, grid, blk, s, t.jobs, g,
                      t.lists, c.count, ws);
    }
    constexpr bool REAL = KC == 1;
    const char *name = REAL ? "kb_sample_sym_chi2" : "kb_sample_chi2";
    if (grads)
        return launch(name, kb_sample_chi2<T, REAL, true>, grid, blk, s, t.jobs, g, t.lists, c.count, ws);
    if (c.multi)
        return launch(name, kb_sample_chi2<T, REAL, false, true>, grid, blk, s, t.jobs, g, t.lists,
                      c.count, ws);
    return launch(name, kb_sample_chi2<T, REAL, false>, grid, blk, s, t.jobs, g, t.lists, c.count, ws);
}

template <typename T>
static int batch_sample_any(const BatchPlan::SClass &c, bool grads, const BatchTables &t,
                            char *ws, hipStream_t s) {
    switch (c.kc) {
        case 0: return batch_sample<T, 0>(c, grads, t, ws, s);
        case 1: return batch_sample<T, 1>(c, grads, t, ws, s);
        case 3: return batch_sample<T, 3>(c, grads, t, ws, s);
        case 4: return batch_sample<T, 4>(c, grads, t, ws, s);
        case 5: return batch_sample<T, 5>(c, grads, t, ws, s);
        default: return fail(GAL_ERR_UNSUPPORTED, "sample class %d", c.kc);
    }
}

static int exec_plan(const BatchPlan &P, const BatchTables &t, char *ws, double *chi2, hipStream_t s) {
    int rc = launch("kb_prepare", kb_prepare, dim3((P.n + 63) / 64), dim3(64), s, t.jobs, P.n,
                    (Control *)ws);
    if (rc) return rc;
    if (P.zero_end > P.zero_begin) {
        const int64_t zb = (int64_t)(P.zero_end - P.zero_begin);
        rc = launch("k_zero", k_zero16, dim3(zero_grid(zb)), dim3(256), s, (void *)(ws + P.zero_begin),
                    zb, (void *)nullptr, (int64_t)0);
        if (rc) return rc;
    }
    for (const auto &f : P.fgroups) {
        rc = f.prec == 8 ? batch_fft<double>(f, t, ws, s) : batch_fft<float>(f, t, ws, s);
        if (rc) return rc;
    }
    for (const auto &c : P.sclasses) {
        rc = c.prec == 8 ? batch_sample_any<double>(c, P.grads, t, ws, s)
                         : batch_sample_any<float>(c, P.grads, t, ws, s);
        if (rc) return rc;
    }
    rc = launch("kb_reduce", kb_reduce, dim3(P.n), dim3(REDUCE_NT), s, t.jobs, P.n, t.groups,
                t.job_group, ws, chi2);
    if (rc) return rc;
    for (const auto &f : P.agroups) {
        rc = f.prec == 8 ? batch_adj<double>(f, t, ws, s) : batch_adj<float>(f, t, ws, s);
        if (rc) return rc;
    }
    return GAL_OK;
}

int gal_batch_create(const gal_job *jobs, int n, gal_batch **out) {
    if (!out) return fail(GAL_ERR_NULL, "NULL argument");
    *out = nullptr;
    int rc = ensure_init();
    if (rc) return rc;
    gal_batch *b = new gal_batch();
    rc = plan_batch(jobs, n, nullptr, 256, b->plan);
    if (rc) {
        delete b;
        return rc;
    }
    GAL_HIP(hipGetDevice(&b->device));
    if (hipMalloc(&b->dtab, b->plan.table_bytes) != hipSuccess) {
        delete b;
        return fail(GAL_ERR_WORKSPACE, "out of device memory for a batch table");
    }
    const std::vector<char> h = table_image(b->plan);
    if (hipMemcpy(b->dtab, h.data(), h.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(b->dtab);
        delete b;
        return fail(GAL_ERR_HIP, "batch table upload failed");
    }
    *out = b;
    return GAL_OK;
}

size_t gal_batch_workspace_bytes(const gal_batch *b) { return b ? b->plan.ws_need : 0; }

int gal_batch_info(const gal_batch *b, int *n_jobs, int *n_fft_groups, int *n_sample_groups) {
    if (!b) return fail(GAL_ERR_NULL, "NULL batch");
    if (n_jobs) *n_jobs = b->plan.n;
    if (n_fft_groups) *n_fft_groups = (int)b->plan.fgroups.size();
    if (n_sample_groups) *n_sample_groups = (int)b->plan.groups.size();
    return GAL_OK;
}

int gal_batch_chi2(const gal_batch *b, double *chi2, void *ws, size_t ws_bytes_, void *stream) {
    if (!b || !chi2 || !ws) return fail(GAL_ERR_NULL, "NULL argument");
    if (ws_bytes_ < b->plan.ws_need)
        return fail(GAL_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes_, b->plan.ws_need);
    return exec_plan(b->plan, tables_at(b->plan, b->dtab), (char *)ws, chi2, (hipStream_t)stream);
}

int gal_batch_destroy(gal_batch *b) {
    if (!b) return GAL_OK;
    int cur = 0;
    GAL_HIP(hipGetDevice(&cur));
    if (cur != b->device) GAL_HIP(hipSetDevice(b->device));
    hipError_t e = hipFree(b->dtab);
    if (cur != b->device) (void)hipSetDevice(cur);
    delete b;
    if (e != hipSuccess) return fail(GAL_ERR_HIP, "hipFree: %s", hipGetErrorString(e));
    return GAL_OK;
}

// one-shot execution: the table travels in the workspace (after its control block)
size_t gal_batch_exec_workspace_bytes(const gal_job *jobs, int n, void *const *grads) {
    BatchPlan P;
    if (plan_batch(jobs, n, grads, 256, P) != GAL_OK) return 0;
    return align256(256 + P.table_bytes) + (P.ws_need - 256);
}

int gal_batch_exec(const gal_job *jobs, int n, double *chi2, void *const *grads, void *ws,
                   size_t ws_bytes_, void *stream) {
    if (!chi2 || !ws) return fail(GAL_ERR_NULL, "NULL argument");
    int rc = ensure_init();
    if (rc) return rc;
    BatchPlan P;
    rc = plan_batch(jobs, n, grads, 256, P);
    if (rc) return rc;
    const size_t tab = align256(256 + P.table_bytes) - 256;  // table after the control block
    const size_t need = P.ws_need + tab;
    if (ws_bytes_ < need) return fail(GAL_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes_, need);
    // shift the data layout past the table
    for (auto &j : P.jobs) {
        j.part_off += tab;
        j.spec_off += tab;
        if (j.grad) {
            j.a_off += tab;
            if (j.kind == 1) j.gi_off += tab;
        }
    }
    P.zero_begin += tab;
    P.zero_end += tab;
    hipStream_t s = (hipStream_t)stream;
    // the table is copied from host memory that is freed on return: a copy
    // captured into a graph would read it at every replay
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    GAL_HIP(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(GAL_ERR_UNSUPPORTED,
                    "gal_batch_exec cannot be captured into a graph (its plan is made at the "
                    "call): capture gal_batch_chi2 of a gal_batch_create plan instead");
    char *w = (char *)ws;
    const std::vector<char> h = table_image(P);
    // a copy from pageable memory: HIP stages the source before returning
    GAL_HIP(hipMemcpyAsync(w + 256, h.data(), h.size(), hipMemcpyHostToDevice, s));
    return exec_plan(P, tables_at(P, w + 256), w, chi2, s);
}

// ---- autotuning ----------------------------------------------------------
int gal_autotune_d(int Nxy, double frac, void *stream, int *chosen, double *times_ms) {
    return autotune<double>(Nxy, frac, stream, chosen, times_ms);
}
int gal_autotune_f(int Nxy, double frac, void *stream, int *chosen, double *times_ms) {
    return autotune<float>(Nxy, frac, stream, chosen, times_ms);
}
int gal_tune_get(int precision, int Nxy, int *chosen) {
    if (!chosen) return fail(GAL_ERR_NULL, "NULL chosen");
    if (!pow2_in_range(Nxy) || (precision != 8 && precision != 4))
        return fail(GAL_ERR_SIZE, "bad precision or Nxy");
    for (int k = 0; k < NKIND; ++k)
        chosen[k] = precision == 8 ? chosen_var<double>(Nxy, k) : chosen_var<float>(Nxy, k);
    return GAL_OK;
}
int gal_tune_set(int precision, int Nxy, const int *chosen) {
    if (!chosen) return fail(GAL_ERR_NULL, "NULL chosen");
    if (!pow2_in_range(Nxy) || (precision != 8 && precision != 4))
        return fail(GAL_ERR_SIZE, "bad precision or Nxy");
    for (int k = 0; k < NKIND; ++k)
        if (chosen[k] < -1 || chosen[k] >= NVAR) return fail(GAL_ERR_SIZE, "variant out of range");
    (void)chosen_var<double>(Nxy, 0);  // initialise the table
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int k = 0; k < NKIND; ++k) g_choice[precision == 8 ? 0 : 1][log2i(Nxy)][k] = chosen[k];
    return GAL_OK;
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

// ---- stage-handoff probe ----------------------------------------------------
// Every block writes its slice of a stage output, then publishes it with one
// agent-scope atomic on a counter (MODE 0: none, 1: relaxed, 2: release,
// 3: acquire-release).  Nothing waits on the counter, so every block exits.
constexpr int PROBE_NT = 256, PROBE_PER_THREAD = 4;
template <int MODE>
__global__ __launch_bounds__(PROBE_NT) void k_stage_probe(double *__restrict__ out,
                                                          unsigned int *ctr) {
    double *o = out + (size_t)blockIdx.x * (PROBE_NT * PROBE_PER_THREAD);
#pragma unroll
    for (int k = 0; k < PROBE_PER_THREAD; ++k)
        o[threadIdx.x + PROBE_NT * k] = (double)(blockIdx.x + k);
    __syncthreads();
    if (threadIdx.x == 0) {
        if constexpr (MODE == 1)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else if constexpr (MODE == 2)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else if constexpr (MODE == 3)
            __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
}

size_t gal_probe_stage_bytes(int blocks) {
    if (blocks < 1 || blocks > 65536) return 0;
    return 256 + (size_t)blocks * PROBE_NT * PROBE_PER_THREAD * sizeof(double);
}

int gal_probe_stage(int mode, int blocks, void *ws, size_t ws_bytes_, void *stream) {
    if (!ws) return fail(GAL_ERR_NULL, "workspace is NULL");
    if (mode < 0 || mode > 3) return fail(GAL_ERR_SIZE, "probe mode %d", mode);
    const size_t need = gal_probe_stage_bytes(blocks);
    if (need == 0) return fail(GAL_ERR_SIZE, "probe blocks %d", blocks);
    if (ws_bytes_ < need) return fail(GAL_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes_, need);
    int rc = ensure_init();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    unsigned int *ctr = (unsigned int *)ws;
    double *out = (double *)((char *)ws + 256);
    const dim3 grid(blocks), blk(PROBE_NT);
    switch (mode) {
        case 0: return launch("k_stage_probe<0>", k_stage_probe<0>, grid, blk, s, out, ctr);
        case 1: return launch("k_stage_probe<1>", k_stage_probe<1>, grid, blk, s, out, ctr);
        case 2: return launch("k_stage_probe<2>", k_stage_probe<2>, grid, blk, s, out, ctr);
        default: return launch("k_stage_probe<3>", k_stage_probe<3>, grid, blk, s, out, ctr);
    }
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
