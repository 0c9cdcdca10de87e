/*
 * galario_hip.h -- C ABI of an MI355X (gfx950) implementation of the
 * visibility / chi-square path of Tazzari, Beaujean & Testi, "GALARIO: a GPU
 * accelerated library for analysing radio interferometer observations"
 * (MNRAS 2018, arXiv:1709.06999).
 *
 * The library turns a model image, or a radial profile swept into one, into
 * synthetic visibilities at arbitrary (u, v) points, and the weighted
 * chi-square against observed visibilities (Sec. 2.2 lists the calls; Sec. 4,
 * Fig. flow, the steps: create image -> rotate -> shift/FFT/shift ->
 * interpolate -> translate -> reduce chi^2).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units (Sec. 2.2): angles (dxy, Rmin, dR, PA, inc, dRA, dDec) in radians;
 *    u, v in wavelengths; images in Jy/pixel; profiles in Jy/sr; visibilities
 *    in Jy; weights w = 1/sigma^2 in Jy^-2.
 *  - Image layout: Nxy x Nxy, row-major, row 0 = North, column 0 = East,
 *    pixel (r, c) centred at x = (Nxy/2 - c) dxy, y = (Nxy/2 - r) dxy;
 *    the origin (x, y) = (0, 0) is pixel (Nxy/2, Nxy/2) (Sec. 2.2, App. D).
 *  - Transform convention (App. D): V(u, v) = sum_pixels I exp(+2 pi i (u x + v y)),
 *    sampled by bilinear interpolation of the real-to-complex half spectrum
 *    (Sec. 3.4) after rotating (u, v) by PA (Sec. 3.3) and mirroring points
 *    with u' < 0; the offset (dRA, dDec) multiplies V by
 *    exp(+2 pi i (u dRA + v dDec)) (Sec. 3.3).  The body text of Sec. 3.1
 *    writes the conjugate convention.
 *  - inc: for *Profile the sweep stretches x by 1/cos(inc) (Sec. 2.2).  For
 *    *Image a non-zero inc deprojects the rotated u' <- u' cos(inc) and
 *    scales V by cos(inc), the transform of the image stretched the same way
 *    (extension; inc = 0 is the paper's *Image).
 *  - Nxy must be a power of two, 16 <= Nxy <= 16384 for sweep, sample*,
 *    chi2* and the dataset calls (the sizes of the paper's timing tables,
 *    Sec. 6.1 and App. B), 16 <= Nxy <= 8192 for gradients, geometry
 *    gradients, batches, the autotuner and gal_spectrum_* /
 *    gal_sample_spectrum_*.  At 16384 a full-length FP64 column does not fit
 *    in one workgroup's LDS: swept profiles then use half-length transforms of
 *    even sequences in both passes and images a two-launch column pass, whose
 *    spectrum takes a second region of the workspace.  A uv point is usable
 *    when all four nodes of its bilinear stencil lie on the half spectrum:
 *    0 <= floor(|u'|/du) <= Nxy/2 - 1 and -Nxy/2 <= floor(v'/du) <= Nxy/2 - 2,
 *    du = 1/(Nxy dxy).  Calls on raw uv arrays check this per point on the
 *    device: offending points give NaN and raise the workspace status flag
 *    (gal_read_status).  Calls on a dataset check it on the host before any
 *    launch from the dataset's rho_max (GAL_ERR_UV_RANGE when
 *    rho_max >= (Nxy/2 - 1) du).
 *  - Precision: suffix _d = double arrays, _f = float arrays.  Scalars are
 *    always double; uv geometry and the chi^2 accumulation run in FP64 in
 *    both variants; the image, the FFT and the visibilities use the array
 *    type (Sec. 2.1: identical interfaces for single and double precision).
 *  - Pointers: every array argument is a caller-owned DEVICE pointer on the
 *    current HIP device, contiguous, not retained after return; arrays of
 *    complex values are interleaved (re, im).  chi2 outputs are device
 *    doubles.  `stream` is a hipStream_t (NULL = default stream); all work is
 *    enqueued on it and the calls return without synchronising.
 *  - Workspace: `ws` is caller-owned device memory of at least
 *    gal_workspace_bytes_{d,f}(Nxy, M) bytes whose first 256 bytes were zeroed
 *    once (gal_workspace_init).  Calls sharing one workspace must be ordered
 *    (same stream); the library itself allocates nothing in these calls.
 *  - Errors: every call returns GAL_OK or a negative GAL_ERR_* code, checked
 *    on the host before anything is enqueued (no output is written on an
 *    error); gal_last_error() gives a message for the calling thread.
 */
#ifndef GALARIO_HIP_H
#define GALARIO_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GAL_OK               0
#define GAL_ERR_NULL        (-1)  /* a required pointer is NULL */
#define GAL_ERR_SIZE        (-2)  /* Nxy outside the sizes above, Nr < 2, M < 0 */
#define GAL_ERR_UV_RANGE    (-3)  /* dataset rho_max outside the half spectrum */
#define GAL_ERR_SCALAR      (-4)  /* dxy < 1e-100, dR <= 0, Rmin < 0, cos(inc) <= 0, non-finite */
#define GAL_ERR_WORKSPACE   (-5)  /* workspace too small / out of memory */
#define GAL_ERR_HIP         (-6)  /* a HIP runtime call failed */
#define GAL_ERR_UNSUPPORTED (-7)  /* e.g. dataset precision differs from the call */

/* ---- library ---------------------------------------------------------- */
const char *gal_version(void);
/* Message describing the last error returned on the calling thread. */
const char *gal_last_error(void);
/* Prepare `device` (upload the twiddle tables).  Optional: every call does it
 * on first use; call it before capturing calls into a HIP graph. */
int gal_init(int device);

/* Bytes of workspace needed by any call with this image size and point
 * count (plain and dataset calls, sample and chi2). */
size_t gal_workspace_bytes_d(int Nxy, int64_t M);
size_t gal_workspace_bytes_f(int Nxy, int64_t M);
/* Zero the control block (first 256 bytes) of a workspace, on `stream`. */
int gal_workspace_init(void *ws, size_t ws_bytes, void *stream);
/* Synchronise `stream`, return the workspace status flag in *status
 * (0 = fine; bit 1: some uv point fell outside the half spectrum; bit 2: a
 * batch job's geometry row failed its checks) and clear it. */
int gal_read_status(void *ws, void *stream, int *status);

/* ---- the paper's calls (Sec. 2.2) on raw device arrays ---------------- */

/* sweep: image[Nxy*Nxy] from the radial profile I[Nr] on r_j = Rmin + j dR:
 * linear interpolation in radius rho = sqrt((x/cos inc)^2 + y^2), 0 outside
 * [Rmin, Rmin + (Nr-1) dR], centre pixel = the first segment extrapolated to
 * rho = 0, times dxy^2 (Sec. 2.2, Sec. 4 "Create image", App. D). */
int gal_sweep_d(const double *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                double inc, double *image, void *stream);
int gal_sweep_f(const float *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                double inc, float *image, void *stream);

/* sampleImage: vis[2M] = V at the M points (Sec. 2.2, Sec. 3.3, Sec. 3.4). */
int gal_sampleImage_d(const double *image, int Nxy, double dxy, const double *u,
                      const double *v, int64_t M, double PA, double dRA, double dDec,
                      double inc, double *vis, void *ws, size_t ws_bytes, void *stream);
int gal_sampleImage_f(const float *image, int Nxy, double dxy, const float *u,
                      const float *v, int64_t M, double PA, double dRA, double dDec,
                      double inc, float *vis, void *ws, size_t ws_bytes, void *stream);

/* sampleProfile: sweep then sampleImage, without materialising the image. */
int gal_sampleProfile_d(const double *I, int Nr, double Rmin, double dR, int Nxy,
                        double dxy, const double *u, const double *v, int64_t M,
                        double inc, double PA, double dRA, double dDec, double *vis,
                        void *ws, size_t ws_bytes, void *stream);
int gal_sampleProfile_f(const float *I, int Nr, double Rmin, double dR, int Nxy,
                        double dxy, const float *u, const float *v, int64_t M,
                        double inc, double PA, double dRA, double dDec, float *vis,
                        void *ws, size_t ws_bytes, void *stream);

/* chi2Image: *chi2 = sum_k w_k |Vobs_k - V_k|^2 (Sec. 3.1, Eq. def.chi.square),
 * reduced on the device in a fixed order (bitwise repeatable). */
int gal_chi2Image_d(const double *image, int Nxy, double dxy, const double *u,
                    const double *v, const double *re, const double *im, const double *w,
                    int64_t M, double PA, double dRA, double dDec, double inc,
                    double *chi2, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Image_f(const float *image, int Nxy, double dxy, const float *u,
                    const float *v, const float *re, const float *im, const float *w,
                    int64_t M, double PA, double dRA, double dDec, double inc,
                    double *chi2, void *ws, size_t ws_bytes, void *stream);

/* chi2Profile: sweep + chi2Image; only the profile is read (Sec. 4). */
int gal_chi2Profile_d(const double *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                      const double *u, const double *v, const double *re, const double *im,
                      const double *w, int64_t M, double inc, double PA, double dRA,
                      double dDec, double *chi2, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Profile_f(const float *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                      const float *u, const float *v, const float *re, const float *im,
                      const float *w, int64_t M, double inc, double PA, double dRA,
                      double dDec, double *chi2, void *ws, size_t ws_bytes, void *stream);

/* ---- separately callable steps (Sec. 4: every operation is accessible) -- */

/* spectrum: the half spectrum G[Nxy][Nxy/2+1] (interleaved complex) of the
 * image with its origin moved to pixel (Nxy/2, Nxy/2):
 * G[p][q] = sum_{r,c} img[r][c] exp(-2 pi i (p (r - Nxy/2) + q (c - Nxy/2)) / Nxy),
 * row p holds frequency p - Nxy [p >= Nxy/2]  (Sec. 4: shift -> FFT -> shift). */
int gal_spectrum_d(const double *image, int Nxy, double *spec, void *ws, size_t ws_bytes,
                   void *stream);
int gal_spectrum_f(const float *image, int Nxy, float *spec, void *ws, size_t ws_bytes,
                   void *stream);
/* sample_spectrum: sample a half spectrum in the layout above at the M points
 * (rotation, mirror, bilinear, deprojection, phase; Sec. 3.3, Sec. 3.4). */
int gal_sample_spectrum_d(const double *spec, int Nxy, double dxy, const double *u,
                          const double *v, int64_t M, double PA, double dRA, double dDec,
                          double inc, double *vis, void *ws, size_t ws_bytes, void *stream);
int gal_sample_spectrum_f(const float *spec, int Nxy, double dxy, const float *u,
                          const float *v, int64_t M, double PA, double dRA, double dDec,
                          double inc, float *vis, void *ws, size_t ws_bytes, void *stream);

/* ---- device-resident datasets ------------------------------------------
 * A dataset is an observation (u, v, Re Vobs, Im Vobs, w)[M] copied once into
 * library-owned device memory, with rho_max = max_k sqrt(u_k^2 + v_k^2)
 * (PA-independent).  Calls on a dataset read no observation from the host,
 * check the uv range on the host, and only transform the part of the half
 * spectrum that the points can reach (|u'|, |v'| <= rho_max): the samples are
 * the same as on the full spectrum.  `precision` of the arrays is fixed at
 * creation (_d: double, _f: float).  re/im/w may be NULL for a dataset used
 * only by sample calls; an empty dataset (M = 0) counts as holding (no)
 * observations, and its chi^2 is 0.  Creation allocates and synchronises
 * `stream`. */
typedef struct gal_dataset gal_dataset;
int gal_dataset_create_d(const double *u, const double *v, const double *re,
                         const double *im, const double *w, int64_t M, void *stream,
                         gal_dataset **out);
int gal_dataset_create_f(const float *u, const float *v, const float *re,
                         const float *im, const float *w, int64_t M, void *stream,
                         gal_dataset **out);
int gal_dataset_destroy(gal_dataset *ds);
/* M, rho_max and the precision (8 = double, 4 = float) of a dataset. */
int gal_dataset_info(const gal_dataset *ds, int64_t *M, double *rho_max, int *precision);

/* Part of the half spectrum a call on a dataset transforms for this image:
 * columns q in [0, *Q) and rows p~ in [-*P, *P] (frequencies in units of
 * du = 1/(Nxy dxy)); *Q = Nxy/2 + 1, *P = Nxy/2 is the whole spectrum. */
int gal_dataset_geometry(const gal_dataset *ds, int Nxy, double dxy, int *Q, int *P);

int gal_chi2Image_ds_d(const gal_dataset *ds, const double *image, int Nxy, double dxy,
                       double PA, double dRA, double dDec, double inc, double *chi2,
                       void *ws, size_t ws_bytes, void *stream);
int gal_chi2Image_ds_f(const gal_dataset *ds, const float *image, int Nxy, double dxy,
                       double PA, double dRA, double dDec, double inc, double *chi2,
                       void *ws, size_t ws_bytes, void *stream);
int gal_chi2Profile_ds_d(const gal_dataset *ds, const double *I, int Nr, double Rmin,
                         double dR, int Nxy, double dxy, double inc, double PA, double dRA,
                         double dDec, double *chi2, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Profile_ds_f(const gal_dataset *ds, const float *I, int Nr, double Rmin,
                         double dR, int Nxy, double dxy, double inc, double PA, double dRA,
                         double dDec, double *chi2, void *ws, size_t ws_bytes, void *stream);

/* chi2Profile on a dataset with the library's own scratch workspace: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The same result as
 * gal_chi2Profile_ds_d; the call allocates nothing.  The workspace is a
 * static device array of GAL_SCRATCH_BYTES on every device the library runs
 * on, held until the process ends; a call needing more
 * (gal_workspace_bytes_d(Nxy, M) > GAL_SCRATCH_BYTES: Nxy <= 2048 fits up to
 * M of about 4e9 points, Nxy >= 4096 never fits) returns GAL_ERR_WORKSPACE
 * with nothing enqueued.  Its set-up (twiddle tables, the scratch address, its
 * status word cleared) runs in gal_init(device) or else on the first call on
 * a device: call gal_init before capturing.  Every call on one device shares
 * that device's scratch: calls on different streams that overlap race and
 * must be ordered by the caller. */
#define GAL_SCRATCH_BYTES (64u << 20)
int gal_chi2Profile_ds_scratch_d(const gal_dataset *ds, const double *I, int Nr, double Rmin,
                                 double dR, int Nxy, double dxy, double inc, double PA,
                                 double dRA, double dDec, double *chi2, void *stream);
int gal_sampleImage_ds_d(const gal_dataset *ds, const double *image, int Nxy, double dxy,
                         double PA, double dRA, double dDec, double inc, double *vis,
                         void *ws, size_t ws_bytes, void *stream);
int gal_sampleImage_ds_f(const gal_dataset *ds, const float *image, int Nxy, double dxy,
                         double PA, double dRA, double dDec, double inc, float *vis,
                         void *ws, size_t ws_bytes, void *stream);
int gal_sampleProfile_ds_d(const gal_dataset *ds, const double *I, int Nr, double Rmin,
                           double dR, int Nxy, double dxy, double inc, double PA,
                           double dRA, double dDec, double *vis, void *ws, size_t ws_bytes,
                           void *stream);
int gal_sampleProfile_ds_f(const gal_dataset *ds, const float *I, int Nr, double Rmin,
                           double dR, int Nxy, double dxy, double inc, double PA,
                           double dRA, double dDec, float *vis, void *ws, size_t ws_bytes,
                           void *stream);

/* ---- gradients (not in the paper) ----------------------------------------
 * chi^2 and its gradient with respect to the image pixels (grad[Nxy*Nxy],
 * layout of the image) or to the profile values (grad[Nr]).  chi^2 is exactly
 * quadratic in both, and the gradient is the exact transpose of the forward
 * map: the residuals w_k (Vobs_k - V_k) scattered onto the bilinear nodes of
 * the half spectrum (with the phase and mirror of each point), the
 * transposed transforms, and for profiles the transposed sweep
 *   dchi2/dI_j = sum_pixels dchi2/dimg * dimg/dI_j.
 * The scatter and the profile bins use floating-point atomics, so gradients
 * are not bitwise repeatable (chi^2 is).  Profile gradients need Nr <= 8192.
 * Workspace: gal_grad_workspace_bytes_* (first 256 bytes zeroed once). */
size_t gal_grad_workspace_bytes_d(int Nxy, int64_t M, int Nr);
size_t gal_grad_workspace_bytes_f(int Nxy, int64_t M, int Nr);
int gal_chi2Image_grad_d(const double *image, int Nxy, double dxy, const double *u,
                         const double *v, const double *re, const double *im, const double *w,
                         int64_t M, double PA, double dRA, double dDec, double inc,
                         double *chi2, double *grad, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Image_grad_f(const float *image, int Nxy, double dxy, const float *u,
                         const float *v, const float *re, const float *im, const float *w,
                         int64_t M, double PA, double dRA, double dDec, double inc,
                         double *chi2, float *grad, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Profile_grad_d(const double *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                           const double *u, const double *v, const double *re, const double *im,
                           const double *w, int64_t M, double inc, double PA, double dRA,
                           double dDec, double *chi2, double *grad, void *ws, size_t ws_bytes,
                           void *stream);
int gal_chi2Profile_grad_f(const float *I, int Nr, double Rmin, double dR, int Nxy, double dxy,
                           const float *u, const float *v, const float *re, const float *im,
                           const float *w, int64_t M, double inc, double PA, double dRA,
                           double dDec, double *chi2, float *grad, void *ws, size_t ws_bytes,
                           void *stream);
int gal_chi2Image_grad_ds_d(const gal_dataset *ds, const double *image, int Nxy, double dxy,
                            double PA, double dRA, double dDec, double inc, double *chi2,
                            double *grad, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Image_grad_ds_f(const gal_dataset *ds, const float *image, int Nxy, double dxy,
                            double PA, double dRA, double dDec, double inc, double *chi2,
                            float *grad, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Profile_grad_ds_d(const gal_dataset *ds, const double *I, int Nr, double Rmin,
                              double dR, int Nxy, double dxy, double inc, double PA, double dRA,
                              double dDec, double *chi2, double *grad, void *ws, size_t ws_bytes,
                              void *stream);
int gal_chi2Profile_grad_ds_f(const gal_dataset *ds, const float *I, int Nr, double Rmin,
                              double dR, int Nxy, double dxy, double inc, double PA, double dRA,
                              double dDec, double *chi2, float *grad, void *ws, size_t ws_bytes,
                              void *stream);

/* ---- gradient with respect to the geometry (not in the paper) --------------
 * chi^2 and d chi^2 / d (PA, dRA, dDec, inc) of chi2Image / chi2Profile on a
 * dataset: *chi2 (device double) and dgeo[4] (device doubles, in that order).
 * Offsets enter through the phase (dV/d dRA = 2 pi i u V); PA through the
 * rotated, mirrored grid coordinates and the bilinear interpolant's
 * derivative inside its cell (it jumps across cell edges); the inclination of
 * an image through the u' cos(inc) deprojection and flux factor (A-15), that
 * of a swept profile through the image itself: its derivative
 * (x / cos inc)^2 tan(inc) / rho * dI/drho * dxy^2 is transformed by the same
 * passes and sampled at the same stencils.  Workspace:
 * gal_geograd_workspace_bytes (256-byte aligned, first 256 bytes zeroed once).
 * Errors as the chi^2 calls on datasets. */
size_t gal_geograd_workspace_bytes_d(int Nxy, int64_t M);
size_t gal_geograd_workspace_bytes_f(int Nxy, int64_t M);
int gal_chi2Image_geograd_ds_d(const gal_dataset *ds, const double *image, int Nxy, double dxy,
                               double PA, double dRA, double dDec, double inc, double *chi2,
                               double *dgeo, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Image_geograd_ds_f(const gal_dataset *ds, const float *image, int Nxy, double dxy,
                               double PA, double dRA, double dDec, double inc, double *chi2,
                               double *dgeo, void *ws, size_t ws_bytes, void *stream);
int gal_chi2Profile_geograd_ds_d(const gal_dataset *ds, const double *I, int Nr, double Rmin,
                                 double dR, int Nxy, double dxy, double inc, double PA,
                                 double dRA, double dDec, double *chi2, double *dgeo, void *ws,
                                 size_t ws_bytes, void *stream);
int gal_chi2Profile_geograd_ds_f(const gal_dataset *ds, const float *I, int Nr, double Rmin,
                                 double dR, int Nxy, double dxy, double inc, double PA,
                                 double dRA, double dDec, double *chi2, double *dgeo, void *ws,
                                 size_t ws_bytes, void *stream);

/* ---- image size (Sec. 3.4, criteria (i), (iia), (iib)) -------------------
 * Host-side planning from the uv coverage, no device work.  The uv cell is
 * du = rho_min / (Gamma f_min) -- the image spans f_min times the largest
 * recoverable scale Gamma / rho_min, criterion (iia) -- or, with a primary-beam
 * FWHM PB > 0 [rad], du = 1 / PB (criterion (iib)).  Nxy is the smallest power
 * of two with Nxy du / 2 >= f_max rho_max (criterion (i)) and dxy = 1 / (Nxy du)
 * [rad].  Typical values: f_min = 5, f_max = 2.5, Gamma = 0.6 (they reproduce
 * the paper's table of ALMA and VLA configurations).  Errors: GAL_ERR_SCALAR
 * for f_max <= 2, f_min <= 1 or Gamma <= 0 with PB = 0, rho_min = 0 with PB = 0,
 * PB < 0, an empty or non-finite uv range; GAL_ERR_SIZE above 2^30.  The
 * result may exceed the largest image the other calls take (16384).
 * gal_uv_range_*: shortest and longest baseline of HOST arrays u, v [M]
 * (M >= 1).  gal_dataset_image_size: from a dataset's registered range. */
int gal_image_size(double rho_min, double rho_max, double f_min, double f_max, double PB,
                   double Gamma, int *Nxy, double *dxy);
int gal_uv_range_d(const double *u, const double *v, int64_t M, double *rho_min, double *rho_max);
int gal_uv_range_f(const float *u, const float *v, int64_t M, double *rho_min, double *rho_max);
int gal_dataset_image_size(const gal_dataset *ds, double f_min, double f_max, double PB,
                           double Gamma, int *Nxy, double *dxy);
/* As gal_image_size and gal_dataset_image_size, with Nxy the smallest even
 * 2^a 3^b 5^c (not only powers of two) meeting criterion (i): the paper
 * advises powers of two, these sizes run on the forward calls' mixed-radix
 * path up to 8192 and are never larger than the power-of-two answer. */
int gal_image_size_smooth(double rho_min, double rho_max, double f_min, double f_max, double PB,
                          double Gamma, int *Nxy, double *dxy);
int gal_dataset_image_size_smooth(const gal_dataset *ds, double f_min, double f_max, double PB,
                                  double Gamma, int *Nxy, double *dxy);

/* ---- batches: many chi^2 evaluations per launch --------------------------
 * A batch is a fixed list of jobs, planned once.  Jobs with the same
 * precision, kind and image size share the FFT launches; jobs on the same
 * dataset with the same kind and image grid (up to 16 per group) share one
 * pass over the observations, which are then read once for the whole group
 * (the typical case: the walkers of an MCMC ensemble).  At execution the
 * kernels read the current model arrays and geometry from the device pointers
 * in the jobs, so a plan -- and a HIP graph captured from gal_batch_chi2 -- is
 * reused while the caller rewrites those buffers between executions.  The
 * geometry rows are checked on the device at every execution, as the single
 * calls check them on the host (finite PA, inc, dRA, dDec, cos(inc) > 0;
 * profiles: finite Rmin >= 0, dR > 0): a job that fails gets a NaN chi^2
 * (that of its whole scene) and a NaN gradient, and the workspace status
 * flag gets bit 2 (gal_read_status).  Creation checks everything else (like
 * the dataset calls), allocates the batch's device table and synchronises
 * the device.
 *
 * Scenes (Sec. 3.2: a field of several sources is the sum of the sources'
 * visibilities, each placed by its own phase shift).  Jobs with the same
 * nonzero `scene` are the sources of one model: they must use the same
 * dataset and may differ in kind, image size, pixel size and geometry.  The
 * sampling pass sums their visibilities at every point before the residual;
 * chi2[j] of every member is the scene's chi^2, and a member's gradient is
 * d chi^2(scene) / d model of that member.  A member with share = k + 1 reads
 * the spectrum of member k of its scene (same kind, Nxy, dxy) instead of
 * transforming its own model (which may then be NULL): an identical source
 * placed elsewhere costs one more gather and no FFT.  Only its PA, dRA and
 * dDec (and inc, for an image) act; a profile's Rmin, dR and inc are the
 * owner's, being part of the transform.  A sharing job has no gradient
 * output of its own: its part of the gradient is added into the owner's.
 * Datasets without observations (gal_dataset_create_* with re, im, w NULL)
 * are accepted for jobs without gradient: their chi^2 is 0 and `vis` gives
 * the visibilities. */
#define GAL_JOB_IMAGE   0
#define GAL_JOB_PROFILE 1
typedef struct {
    const gal_dataset *ds;  /* observations (with re, im, w) */
    int kind;               /* GAL_JOB_IMAGE or GAL_JOB_PROFILE */
    int Nxy;                /* image side (power of two) */
    double dxy;             /* pixel size [rad] */
    int Nr;                 /* profile samples (profile jobs) */
    const void *model;      /* device: image [Nxy*Nxy] or profile [Nr], dataset precision */
    const double *geo;      /* device: {Rmin, dR, inc, PA, dRA, dDec}; Rmin, dR unused for images */
    int scene;              /* 0: the job alone; > 0: the scene it is a source of */
    int share;              /* 0: own spectrum; k + 1: the spectrum of job k (same scene) */
    void *vis;              /* device, nullable: the scene's model visibilities at the
                               dataset's points in registration order, interleaved
                               (re, im) [2M], dataset precision; written at execution */
} gal_job;
typedef struct gal_batch gal_batch;
int gal_batch_create(const gal_job *jobs, int n, gal_batch **out);
/* Workspace bytes gal_batch_chi2 needs (first 256 bytes zeroed once). */
size_t gal_batch_workspace_bytes(const gal_batch *b);
int gal_batch_info(const gal_batch *b, int *n_jobs, int *n_fft_groups, int *n_sample_groups);
/* chi2[j] (device doubles) for every job; bitwise repeatable. */
int gal_batch_chi2(const gal_batch *b, double *chi2, void *ws, size_t ws_bytes, void *stream);
int gal_batch_destroy(gal_batch *b);
/* One-shot execution of a job list (any mix of kinds, sizes, datasets and
 * precisions), planned on the host at every call; the plan's device table
 * travels in the workspace (copied with hipMemcpyAsync from host memory that
 * may be freed when the call returns), so nothing is allocated.  grads
 * (nullable) holds one gradient output per job (device, dataset precision:
 * image [Nxy*Nxy] or profile [Nr]; NULL = chi^2 only); gradient jobs run the
 * adjoint path of the gradient calls above.  Workspace:
 * gal_batch_exec_workspace_bytes (first 256 bytes zeroed once; 0 on error).
 * The host table is copied from pageable memory, which HIP stages before the
 * call returns; because the plan is made at the call, a stream that is being
 * captured into a graph is refused (GAL_ERR_UNSUPPORTED): capture
 * gal_batch_chi2 of a created batch instead. */
size_t gal_batch_exec_workspace_bytes(const gal_job *jobs, int n, void *const *grads);
int gal_batch_exec(const gal_job *jobs, int n, double *chi2, void *const *grads, void *ws,
                   size_t ws_bytes, void *stream);

/* ---- FFT schedule autotuning -------------------------------------------
 * Every FFT pass exists in NVAR = 3 compiled variants that differ in the
 * values each thread holds (16, 8 or 4: more threads per transform, more
 * waves in flight, more radix passes); for the rows of a swept profile they
 * are the half-length transform of even rows with 8 values, the full-length
 * transform of a row pair with 8, and the half-length one with 4.  gal_autotune_* times all variants of
 * the four passes (rows of an image, columns, rows and columns of a swept
 * profile) for one image size on the current device -- with frac the part of
 * the half spectrum transformed (rho_max / ((Nxy/2 - 1) du), 1 = all) -- and
 * keeps the fastest for later calls in this process; chosen[4] receives the
 * choice and times_ms[4 * 3] (nullable) the average launch time of every
 * variant, -1 where a size has fewer variants.  It allocates and frees
 * scratch memory and synchronises `stream`.
 * gal_tune_get / gal_tune_set read and install choices (precision 8 or 4,
 * variant -1 = built-in default), e.g. from a cache file. */
int gal_autotune_d(int Nxy, double frac, void *stream, int *chosen, double *times_ms);
int gal_autotune_f(int Nxy, double frac, void *stream, int *chosen, double *times_ms);
int gal_tune_get(int precision, int Nxy, int *chosen);
int gal_tune_set(int precision, int Nxy, const int *chosen);

/* ---- per-kernel timing (HIP events on the launch stream) ----------------
 * When enabled, every kernel launch of the library is bracketed by HIP events
 * recorded on its stream.  gal_timing_read synchronises, and for each kernel
 * name fills the total milliseconds and launch count since the last reset;
 * it returns the number of kernel names (at most `cap` are filled). */
int gal_timing_enable(int on);
int gal_timing_reset(void);
int gal_timing_read(int cap, const char **names, double *total_ms, int64_t *launches);

/* Measurement aid: the cost of the device-scope handoff a persistent kernel
 * needs between two stages, which is why the batches run one kernel per stage
 * instead.  Launches k_stage_probe over `blocks` blocks of 256 threads on
 * `stream`: every block writes its 8 KB slice of a stage output, then one
 * thread adds 1 to a counter at agent scope with no atomic (mode 0), a relaxed
 * (1), a release (2) or an acquire-release (3) atomic.  Nothing waits on the
 * counter.  ws: device memory of at least gal_probe_stage_bytes(blocks) bytes,
 * the counter in its first 256 bytes.  GAL_ERR_SIZE for a mode outside [0, 3]
 * or blocks outside [1, 65536], GAL_ERR_WORKSPACE for a smaller ws. */
size_t gal_probe_stage_bytes(int blocks);
int gal_probe_stage(int mode, int blocks, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GALARIO_HIP_H */
