/*
 * simus.h -- C ABI of libsimus, an MI355X (gfx950) implementation of the
 * SIMUS radio-frequency synthesis of D. Garcia, "SIMUS: an open-source
 * simulator for medical ultrasound imaging. Part I: theory & examples".
 *
 * The library computes, for every transmit t, receive element e and
 * frequency bin j, the received element spectrum
 *
 *   X[t][e][j] = S_P(w_j) S_T(w_j) sum_s R_s a[s][t](w_j) B[e][s](w_j)
 *
 * with a = sum over all nu*N sub-elements n of W_{t,e(n)} exp(i w tau_{t,e(n)})
 * G_{n,s} (Eq. 29), B = sum of G over the nu sub-elements of element e
 * (Eqs. 32-33), the sub-element Green's term
 *
 *   G_{n,s}(w) = exp(i (k + i k_a) r) / r * D(theta, k) * delta(y, r, k)
 *
 * (Eqs. 17-20 with the sinc directivity of Eq. 10 and the baffle factors of
 * Eq. 39, the four-Gaussian elevation term of Eqs. 12-18 and the
 * attenuation of Eq. 40), the pulse spectrum of Eq. 25 and the transducer
 * spectrum of Eq. 27 (Eqs. 28 and 34), and then the RF signals by the
 * inverse transform of Eq. 1:
 *
 *   rf[t][e][q] = Re sum_j X[t][e][j] exp(-2 pi i j q / nfft).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - SI units (m, s, Hz); attenuation in dB/cm/MHz.
 * - Scatterers are structure-of-arrays float32: x, y, z, refl.  y may be
 *   NULL, meaning y = 0 for every scatterer (the azimuth plane).
 * - Pointers documented "device" must point to memory of the current HIP
 *   device; "host" pointers are read before the call returns.
 * - The caller owns all buffers.  The library owns a workspace cached per
 *   (device, stream), released by simus_release_workspace().
 * - All device work is enqueued on `hip_stream` (a hipStream_t; NULL = the
 *   null stream).  No entry point synchronises the stream; outputs are
 *   ready when the stream's work completes.  Calls that share a stream are
 *   ordered; calls on different streams use different workspaces.  Calls
 *   on one stream must not be made from several host threads at once
 *   (they share that stream's workspace and staging buffer).
 * - Return value: SIMUS_OK (0) or a negative error code.  Arguments are
 *   validated on the host before any HIP call, so invalid arguments never
 *   reach the GPU.  simus_last_error() gives a message (thread-local).
 * - Probe: linear when radius == 0, Eq. (24) sub-element centroids; convex
 *   when radius > 0 (apex at the origin, centre of curvature at (0, -R),
 *   flat elements of chord pitch, split along their face).  A sub-element
 *   does not radiate behind its face (G = 0 where the local depth <= 0).
 * - Domain of the scatterers.  simus_rf_grid reads host copies and returns
 *   SIMUS_EDOMAIN for a scatterer at depth z <= 0 in front of a linear
 *   array, within 1e-9 m of a sub-element centroid, or with a non-finite
 *   coordinate.  The device entry points (simus_rf_spectrum, simus_rf,
 *   simus_rf_backward, simus_pfield, the plan calls) do not read device
 *   data on the host and return no SIMUS_EDOMAIN: there, a (sub-element,
 *   scatterer) pair with the scatterer at local depth <= 0 in front of the
 *   sub-element's face, or within 1e-9 m of its centroid, has G = 0 (and
 *   dG = 0).  So a scatterer behind every sub-element (z <= 0 before a
 *   linear array) adds exactly nothing to spectra, RF or field, and gets
 *   zero gradients; such scatterers do not widen the per-call elevation
 *   table either, so appending them to a phantom leaves its spectra and RF
 *   bit for bit unchanged when the partition into work items
 *   (options.tile_scat) does not move the other scatterers.  Non-finite
 *   device coordinates are not checked and give undefined results.
 */
#ifndef SIMUS_H
#define SIMUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIMUS_VERSION 201

#define SIMUS_OK 0
#define SIMUS_EINVAL (-1)   /* invalid argument (NULL pointer, bad size, bad parameter) */
#define SIMUS_EDOMAIN (-2)  /* scatterer outside the model's domain (simus_rf_grid only) */
#define SIMUS_ENOMEM (-3)   /* device or pinned host allocation failed */
#define SIMUS_EHIP (-4)     /* a HIP runtime call failed */
#define SIMUS_ETOOBIG (-5)  /* simus_rf_noalloc: the call needs more than its scratch */

typedef enum {
    SIMUS_BAFFLE_SOFT = 0,   /* D = sinc(k b sin t) cos t   (Eq. 39, default) */
    SIMUS_BAFFLE_RIGID = 1,  /* D = sinc(k b sin t)                           */
    SIMUS_BAFFLE_ZETA = 2    /* D = sinc(k b sin t) cos t / (cos t + zeta)    */
} simus_baffle;

/* Transducer array (Fig. 2; Sections II-III, VI). */
typedef struct {
    int32_t n_elements;   /* N >= 1 */
    int32_t baffle;       /* simus_baffle */
    double fc;            /* centre frequency [Hz] > 0 */
    double pitch;         /* element pitch [m] > 0 */
    double width;         /* element width 2b [m], 0 < width <= pitch */
    double height;        /* element height h [m] > 0 */
    double elev_focus;    /* elevation focus R_f [m] > 0, may be +INFINITY */
    double bandwidth;     /* pulse-echo fractional -6 dB bandwidth, 0 < bw < 2 */
    double radius;        /* 0: linear array; > 0: convex radius [m] */
    double zeta;          /* baffle impedance ratio (SIMUS_BAFFLE_ZETA), >= 0 */
} simus_probe;

/* Medium (Section VI-B). */
typedef struct {
    double c;             /* speed of sound [m/s] > 0 */
    double alpha_db;      /* amplitude attenuation [dB/cm/MHz] >= 0 (Eq. 40) */
} simus_medium;

/* Sampling and model options. */
typedef struct {
    double fs;            /* RF sampling frequency [Hz], fs > 2 fc */
    double n_cycles;      /* pulse length n_lambda in wavelengths (Eq. 25) > 0 */
    double spectral_eps;  /* evaluated band: contiguous bins spanning every bin with
                             |S_P S_T| >= eps * max (eps in [0, 1)); 1e-7 typical */
    int32_t nu;           /* sub-elements per element; 0 = Eq. (21) with the
                             shortest wavelength at the upper -6 dB edge */
    int32_t nfft;         /* transform length (even).  simus_rf_grid: 0 = auto;
                             every other entry point requires nfft > 0 */
    int32_t n_t;          /* RF samples returned per channel; 0 = nfft; <= nfft */
    int32_t flags;        /* SIMUS_FLAG_* */
    int32_t n_gauss;      /* Gaussians G of the elevation aperture (Eq. 12) in `gauss`,
                             0..SIMUS_MAX_GAUSS; 0 = the four of Eq. (18) */
    int32_t tile_scat;    /* scatterers per work item; 0 = a default from the
                             problem size (simus_rf_plan_autotune measures) */
    const double* gauss;  /* host [n_gauss][4]: Re A_g, Im A_g, Re B_g, Im B_g of
                             Pi(u) ~ sum_g A_g exp(-B_g u^2) (Eqs. 12-16), finite,
                             Re B_g > 0; read before the call returns (plans keep a
                             copy).  Sets of complex-conjugate pairs (as Eq. 18's)
                             make the aperture real.  NULL when n_gauss = 0 */
} simus_options;

#define SIMUS_MAX_GAUSS 32

#define SIMUS_FLAG_NO_MFMA       1   /* never use the MFMA multi-transmit contraction */
#define SIMUS_FLAG_PERSISTENT    2   /* persistent work-queue launch of the synthesis: the
                                        default on every path (the flag is accepted and has
                                        no further effect) */
#define SIMUS_FLAG_NO_DELTA_TABLE 4  /* evaluate the elevation term directly (no table) */
#define SIMUS_FLAG_2D            8   /* 2-D acoustics (Section V, Eqs. 35-38): Green's term
                                        exp(i (k + i k_a) r) / sqrt(r) D in the x-z plane, no
                                        elevation term, factor 2b (element width) on the two-way
                                        spectrum and sqrt(2b) on the one-way field; y (Y) must
                                        be NULL */
#define SIMUS_FLAG_STATIC       16   /* vector path: one block per work item instead of the
                                        persistent launch (the matrix-core path is always
                                        persistent); results are bitwise the same */
#define SIMUS_FLAG_ALT_SHAPE    32   /* the alternative tile shape.  Matrix-core path: the
                                        kernels with FP32 products that set a pair up every
                                        four bins (more than 64 elements; groups of 16
                                        transmit columns up to 16 transmits, else 32) or six
                                        bins (64 or fewer; groups of 32 columns, or 64 above
                                        32 transmits where they pad no more) instead of the
                                        default split-bf16 ones (every eight bins over groups
                                        of 16 up to 16 transmits, every four bins over groups
                                        of 32 above, or of 64 for 64 or fewer elements and
                                        more than 32 transmits).  Vector path: single
                                        transmits instead of pairs, or pairs instead of
                                        single transmits.  The autotuner tries it.
                                        simus_rf_backward: the other of its two kernels
                                        (matrix-core or vector) where both apply.  The
                                        results agree to rounding order */
#define SIMUS_FLAG_FP32_PRODUCTS 64  /* matrix-core path, default shape: the two
                                        contractions with FP32 matrix-core products (eight
                                        bins per set-up over groups of 16 transmit columns)
                                        instead of products of operands split into bf16 high
                                        and low parts (three bf16 products per real product,
                                        FP32 accumulation: about 2^-16 of each product, 5e-6
                                        relative L2 on RF against the FP32 products).  Also
                                        the matrix-core adjoint's GEMM (up to 8 transmits) */
/* Other bits of options.flags are rejected with SIMUS_EINVAL. */

/* Frequency grid of one call. */
typedef struct {
    int32_t nfft;         /* transform length */
    int32_t n_t;          /* RF samples per channel */
    int32_t j_lo;         /* first evaluated bin (absolute index, w_j = 2 pi j fs / nfft) */
    int32_t n_bins;       /* number of evaluated bins j_lo .. j_lo + n_bins - 1 */
    int32_t nu;           /* sub-elements per element */
    int32_t reserved;
    double df;            /* bin spacing fs / nfft [Hz] */
} simus_grid;

int simus_version(void);
const char* simus_last_error(void);

/* Frequency grid for a call (host only, no GPU).
 *   t_max = 2 r_max / c + max delay + 10 / fc, r_max = largest distance from a
 *   sub-element centroid to a scatterer; nfft = options->nfft if > 0, else
 *   the smallest even 2^a 3^b 5^c >= max(fs t_max, n_t).  Bins j with
 *   1 <= j < nfft/2 and f_j < 2 fc are candidates (S_T(2 wc) = 2^-126,
 *   Eq. 49); the evaluated band is per spectral_eps above.
 * delays: host [n_tx][N] seconds (>= 0; positive = fires later, Eq. 20).
 * x, y, z: host [n_scat] (y may be NULL).  n_scat >= 0.
 * Errors: EINVAL for bad parameters; EDOMAIN if a scatterer lies at depth
 * <= 0 in front of a linear array or within 1e-9 m of a sub-element. */
int simus_rf_grid(const simus_probe* probe, const simus_medium* medium,
                  const simus_options* options, int32_t n_tx, const double* delays,
                  int64_t n_scat, const float* x, const float* y, const float* z,
                  simus_grid* out);

/* Element spectra X (Eqs. 22, 29-34) on the evaluated band.
 * delays, apod: host [n_tx][N] (transmit delays [s] and apodisation W).
 * scat_offsets: host [n_phantoms + 1], non-decreasing, scat_offsets[0] = 0;
 *   phantom p owns scatterers scat_offsets[p] .. scat_offsets[p+1]-1.
 * x, y, z, refl: device [scat_offsets[n_phantoms]] float32 (y may be NULL).
 * spec: device float32 [n_phantoms][n_tx][N][n_bins][2] (re, im).
 * Requires options->nfft > 0 (from simus_rf_grid). */
int simus_rf_spectrum(const simus_probe* probe, const simus_medium* medium,
                      const simus_options* options, int32_t n_tx,
                      const double* delays, const float* apod,
                      int32_t n_phantoms, const int64_t* scat_offsets,
                      const float* x, const float* y, const float* z, const float* refl,
                      float* spec, void* hip_stream);

/* RF signals: the spectra above followed by the inverse transform of Eq. (1).
 * rf: device float32 [n_phantoms][n_tx][N][n_t]. */
int simus_rf(const simus_probe* probe, const simus_medium* medium,
             const simus_options* options, int32_t n_tx,
             const double* delays, const float* apod,
             int32_t n_phantoms, const int64_t* scat_offsets,
             const float* x, const float* y, const float* z, const float* refl,
             float* rf, void* hip_stream);

/* simus_rf without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, grid rules and results as simus_rf (to
 * rounding order; bit for bit when the default work-item partition fits).
 * The workspace is a static device array of the library, 64 MiB per GPU,
 * which the GPU holds from the library's first use there until the process
 * ends; the call allocates nothing (no hipMalloc, hipFree, pinned staging or
 * event).  A call whose workspace would exceed the scratch gets longer
 * work items (fewer partial spectra) until it fits; one that cannot fit even
 * then returns SIMUS_ETOOBIG before any HIP call.  The bound is roughly 2e6
 * spectral values n_phantoms x n_tx x N x n_bins (a 128-element plane wave
 * with 850 bins fits; 21 transmits of it do not).  The host
 * tables (about 20 bytes per work item plus the probe's frames and weights)
 * are copied from pageable host memory with hipMemcpyAsync, which may wait
 * for the stream's earlier work.  Every call on a GPU shares that GPU's
 * scratch, and the scratch keeps the last call's contents: calls that may
 * overlap on one GPU (different streams, or several host threads) race and
 * must be serialised by the caller.  Kernel timing (simus_profile_enable)
 * does not record these calls. */
int simus_rf_noalloc(const simus_probe* probe, const simus_medium* medium,
                     const simus_options* options, int32_t n_tx,
                     const double* delays, const float* apod,
                     int32_t n_phantoms, const int64_t* scat_offsets,
                     const float* x, const float* y, const float* z, const float* refl,
                     float* rf, void* hip_stream);

/* Inverse transform alone: rf[c][q] = Re sum_b spec[c][b] exp(-2 pi i (j_lo + b) q / nfft)
 * for q < n_t.  spec: device [n_chan][n_bins][2]; rf: device [n_chan][n_t]. */
int simus_spectrum_to_rf(int32_t nfft, int32_t n_t, int32_t j_lo, int32_t n_bins,
                         int64_t n_chan, const float* spec, float* rf, void* hip_stream);

/* Adjoint of simus_rf: given drf = dL/drf (device, same layout as rf), the
 * gradients dL/drefl, dL/dx, dL/dy, dL/dz (device [n_scat] each; any may be
 * NULL to skip; dy requires y != NULL or is returned for y = 0).  The
 * Green's terms are recomputed per frequency bin, nothing is stored from the
 * forward pass.  Same grid rules as simus_rf (pass the forward's nfft). */
int simus_rf_backward(const simus_probe* probe, const simus_medium* medium,
                      const simus_options* options, int32_t n_tx,
                      const double* delays, const float* apod,
                      int32_t n_phantoms, const int64_t* scat_offsets,
                      const float* x, const float* y, const float* z, const float* refl,
                      const float* drf, float* drefl, float* dx, float* dy, float* dz,
                      void* hip_stream);

/* Number of frequency intervals N_f of the RMS field (Section VII, host only):
 * dw = 2 pi / max over points and sub-elements of (r / c + delay),
 * N_f = ceil(2 wc / dw).  delays: host [N]; X, Y, Z host [n_pts] (Y may be NULL). */
int simus_pfield_nf(const simus_probe* probe, const simus_medium* medium,
                    const simus_options* options, const double* delays,
                    int64_t n_pts, const float* X, const float* Y, const float* Z,
                    int32_t* n_f);

/* RMS pressure field (Eqs. 22, 28, 41, 42): P_RMS(X) = sqrt(dw sum_{j=0}^{N_f}
 * |P(X, w_j)|^2), w_j = 2 wc j / N_f, dw = 2 wc / N_f, P = S_P sqrt(S_T) *
 * sum_n W e^{i w tau} G_n.  delays, apod: host [N]; X, Y, Z: device [n_pts]
 * (Y may be NULL); p_rms: device [n_pts].  n_f >= 1. */
int simus_pfield(const simus_probe* probe, const simus_medium* medium,
                 const simus_options* options, int32_t n_f,
                 const double* delays, const float* apod,
                 int64_t n_pts, const float* X, const float* Y, const float* Z,
                 float* p_rms, void* hip_stream);

/* Forward plan: simus_rf for a fixed probe, medium, options, transmit
 * sequence (delays, apod) and partition into phantoms, so that repeated
 * syntheses of changing scatterers (Eqs. 29-34 and Eq. 1) pay the host work
 * once.  simus_rf_plan_create validates the arguments as simus_rf does,
 * builds the frequency band, the launch configuration and the work items of
 * the (possibly uneven) phantoms, allocates the plan's own device workspace
 * and uploads its tables on hip_stream, then waits for that upload.
 * has_y: nonzero if executions pass y (y != NULL), zero if y = 0.
 * options->flags apply to every execution (the synthesis is one persistent
 * work-queue launch unless SIMUS_FLAG_STATIC).  *plan is set only on
 * success.  The workspace is the plan's: executions of one plan must be
 * ordered (e.g. one stream); different plans may run concurrently. */
typedef struct simus_rf_plan_s* simus_rf_plan;
int simus_rf_plan_create(const simus_probe* probe, const simus_medium* medium,
                         const simus_options* options, int32_t n_tx,
                         const double* delays, const float* apod,
                         int32_t n_phantoms, const int64_t* scat_offsets,
                         int32_t has_y, void* hip_stream, simus_rf_plan* plan);

/* Enqueues one forward synthesis of the plan on hip_stream: x, y, z, refl
 * (device, scat_offsets[n_phantoms] each; y NULL iff the plan was created
 * without y) -> rf (device [n_phantoms][n_tx][N][n_t]).  Kernel launches
 * only: no allocation, copy or host wait, so the call may be captured into
 * a HIP graph by the caller. */
int simus_rf_plan_execute(simus_rf_plan plan, const float* x, const float* y,
                          const float* z, const float* refl, float* rf, void* hip_stream);

/* As simus_rf_plan_execute, through a HIP graph owned by the plan: the first
 * call for a set of pointers (x, y, z, refl, rf) captures the plan's kernels
 * into a graph (on a stream of the plan's own) and instantiates it; every
 * call then launches that graph on hip_stream.  A call with other pointers
 * captures again.  Results equal simus_rf_plan_execute's bit for bit. */
int simus_rf_plan_graph_launch(simus_rf_plan plan, const float* x, const float* y,
                               const float* z, const float* refl, float* rf,
                               void* hip_stream);

/* Autotuner of a plan's launch shape.  Times the plan's kernels (HIP events
 * on hip_stream) on the given scatterers, laid out as for
 * simus_rf_plan_execute, for two tile shapes (the default rule's and,
 * where it differs, SIMUS_FLAG_ALT_SHAPE's), scatterers per work item from
 * 0.5x to 2x the default and, on the vector path, with and without
 * SIMUS_FLAG_STATIC
 * (a warm-up run each, then the mean of three runs, or one run when a run
 * takes over 50 ms);
 * keeps the fastest configuration in the plan (later executions and graph
 * launches use it; a captured graph is dropped) and returns its
 * options.tile_scat and options.flags in *tile_scat and *flags (either may
 * be NULL).  Waits for the device first (earlier executions of the plan on
 * any stream) and for hip_stream at the end; rf is overwritten; the plan's
 * workspace may be reallocated.  On failure the plan keeps its previous
 * configuration.  The results do not depend on the choice beyond rounding
 * order. */
int simus_rf_plan_autotune(simus_rf_plan plan, const float* x, const float* y,
                           const float* z, const float* refl, float* rf, void* hip_stream,
                           int64_t* tile_scat, int32_t* flags);

/* Process-wide file cache of simus_rf_plan_autotune's choices (native, text,
 * one line per choice: problem class, shape flags, scatterers per item as a
 * multiple of the default rule's count, time).  With a path set, the
 * autotuner first looks up the plan's problem class in the file: the path
 * (matrix-core or vector), sub-elements, elements, transmits, y given or
 * not, elevation table, 2-D, the flags other than SIMUS_FLAG_ALT_SHAPE and
 * SIMUS_FLAG_STATIC, the library version, and the
 * binary logarithms of the bins, scatterers and phantoms.  If a line is
 * there (the last one counts), it applies that choice without timing;
 * otherwise it tunes as described above and appends its choice.  Lines are
 * written whole; several processes may share one file.  path NULL or ""
 * switches the cache off (the default).  The path is copied.
 * Errors: EINVAL for a path longer than 4095 bytes; simus_rf_plan_autotune
 * returns EINVAL if it cannot append to the file (the plan keeps the tuned
 * configuration). */
int simus_tune_cache(const char* path);

/* Number of simus_rf_plan_autotune calls of this process answered from the
 * cache. */
int64_t simus_tune_cache_hits(void);

/* Waits for the device, then frees the plan's graph, stream and workspace.
 * NULL is ignored. */
void simus_rf_plan_destroy(simus_rf_plan plan);

/* Frees every cached workspace (all devices, all streams).  Must not run
 * concurrently with other calls. */
void simus_release_workspace(void);

/* Kernel timing (diagnostics).  While enabled, each kernel launch of the
 * library is bracketed by a pair of HIP events recorded on the launch's
 * stream.  simus_profile_read() waits for the recorded events of one kernel
 * ("synth", "wtable", "finalize", "idft", "dft", "adjoint", "adjoint_reduce",
 * "pfield", or "graph" for a whole plan graph launch) and returns their summed duration [ms] and launch count since
 * the last reset.  Returns SIMUS_EINVAL for an unknown name. */
int simus_profile_enable(int on);
int simus_profile_read(const char* kernel, double* total_ms, int64_t* launches);
void simus_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* SIMUS_H */
