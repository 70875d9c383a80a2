/*
 * pw.h -- C ABI of libpw: pairwise line-of-sight power-spectrum and correlation-function
 * multipole estimators on one AMD Instinct MI355X (gfx950).
 *
 * Method: Philcox & Slepian, "Beyond Yamamoto: Anisotropic Power Spectra and Correlation
 * Functions with Pairwise Lines-of-Sight" (arXiv:2102.08384).
 *   - midpoint P_l(k):  Section 3.3, boxed parity-even estimator (coefficients Phi, Appendix D)
 *   - bisector P_l(k):  Section 5.2, boxed estimator (coefficients B, Appendix F)
 *   - midpoint xi_l(r): Section 4.3, boxed parity-even estimator (coefficients F, Appendix E)
 *   - midpoint, all-parity series (midpoint_parity = 1): Section 3.2 (P_l, coefficients phi,
 *     Appendix B) and Section 4.2 (xi_l, coefficients f, Appendix E), every alpha <= order
 *   - bisector xi_l(r): Section 6, boxed estimator (coefficients B)
 * The density field is w (n_g - alpha_r n_r) (Section 2.1); the estimators are normalised
 * by I = alpha_r sum_r w_r^2 nbar_r with alpha_r = sum w_g / sum w_r, and the shot noise
 * S / I, S = sum_g w_g^2 + alpha_r^2 sum_r w_r^2, is subtracted from the power-spectrum
 * monopole only.
 *
 * Conventions
 *   - Positions are comoving, observer at the coordinate origin.  Mesh nodes sit at
 *     box_origin + n * H, H = box_len / n_mesh, n = 0 .. n_mesh-1 per axis, periodic.
 *   - Every particle must satisfy 0 <= x_i - box_origin_i < box_len on every axis
 *     (PW_ERANGE otherwise; particles are never wrapped).
 *   - Series order K: the parity-even midpoint keeps even alpha <= K, the all-parity midpoint
 *     every alpha <= K, the bisector beta <= K/2 (the beta-th bisector term is O(theta^(2 beta))).
 *   - Multipoles are the even ell = 0, 2, ..., ell_max; outputs are [n_ell][n_bins] row-major.
 *   - k bins: bin b holds the modes with b = floor((|k| - bin_lo) / bin_width),
 *     |k| = (2 pi / box_len) sqrt(n_x^2 + n_y^2 + n_z^2) on the signed FFT index
 *     (n >= n_mesh/2 maps to n - n_mesh); decided in FP64 from the integer |n|^2.
 *     r bins: the same with |r| = H sqrt(n^2) on the minimum-image separation; the zero
 *     separation is in no bin.
 *   - P_l values are shell means (the angular average); xi_l values are shell sums divided
 *     by the bin volume N_a H^3 (N_a grid separations in the bin).
 *
 * Precision: PW_FP32 paints, weights and transforms in FP32 and accumulates every shell
 * sum, normalisation and shot-noise term in FP64 on the GPU; PW_FP64 does everything in FP64.
 *
 * Errors: every call returns PW_OK (0) or a negative code; pw_last_error() gives a message.
 * No exception crosses this ABI.  Outputs are written only on success.
 * Threads: a pw_ctx takes pw_estimate-family calls from one thread at a time and submission
 * calls from one thread at a time; the two may be different threads (see pw_submit).
 */
#ifndef PW_H
#define PW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PW_OK = 0,
  PW_EINVAL = -1,    /* malformed configuration or arguments                     */
  PW_ERANGE = -2,    /* a particle lies outside the box                           */
  PW_ENOMEM = -3,    /* the request does not fit the context's HBM budget         */
  PW_EDEVICE = -4,   /* a HIP runtime call failed                                 */
  PW_EBUSY = -5,     /* the submission queue is full (pw_set_queue_limit)         */
  PW_EAGAIN = -6,    /* ticket still pending (pw_poll)                            */
  PW_ECANCELED = -7  /* ticket was cancelled                                      */
};

enum pw_stat { PW_PK = 0, PW_XI = 1 };
enum pw_los { PW_MIDPOINT = 0, PW_BISECTOR = 1 };
enum pw_assign { PW_CIC = 2, PW_TSC = 3 };
enum pw_prec { PW_FP32 = 0, PW_FP64 = 1 };
enum pw_parity { PW_PARITY_EVEN = 0, PW_PARITY_ALL = 1 };

typedef struct pw_ctx pw_ctx;

/* Estimator configuration (the paper's problem statement: box, mesh, ell_max, series
 * order, line of sight, bins).  Zero-initialise it: later fields default to 0. */
typedef struct {
  int stat;              /* PW_PK or PW_XI                                                */
  int los;               /* PW_MIDPOINT or PW_BISECTOR                                    */
  int assign;            /* PW_CIC or PW_TSC                                              */
  int prec;              /* PW_FP32 or PW_FP64                                            */
  int n_mesh;            /* N, a power of two in [16, 512]                                */
  double box_len;        /* L (same length unit as the positions, e.g. Mpc/h)             */
  double box_origin[3];  /* b0, the corner of the box                                     */
  int ell_max;           /* even, 0..8                                                    */
  int order;             /* series order K, 0..8: even, or any for the all-parity midpoint */
  int compensate;        /* 1: divide every k-space factor by the assignment window W(k)  */
  double bin_lo;         /* lower edge of bin 0 (k in 1/length, r in length)              */
  double bin_width;      /* > 0                                                           */
  int n_bins;            /* 1..4096                                                       */
  int midpoint_parity;   /* midpoint series: 0 parity-even (Sections 3.3, 4.3: even alpha, */
                         /* coefficients Phi, F), 1 all-parity (Sections 3.2, 4.2: every   */
                         /* alpha <= order, coefficients phi, f); ignored for the bisector */
  int memory_lean;       /* bisector P_l: 1 = forward transforms in small groups of fields  */
                         /* through group-sized work buffers (about a quarter of the device */
                         /* memory at 512^3, same results bit for bit); ignored elsewhere   */
} pw_config;

/* A catalog: n particles as interleaved (x, y, z, w) records of dtype (PW_FP32 / PW_FP64).
 * nbar (n values of the same dtype, or NULL) is the expected number density at each
 * particle; it is read for the randoms only, to form I.  Pointers are host memory when
 * on_device == 0 and device memory of the context's GPU when on_device == 1.  The caller
 * owns the memory; the library never frees or retains it past the call (pw_estimate) or
 * past the ticket's completion (pw_submit).
 * Device memory must hold its final values when the call is made: the library reads it on
 * its own streams (and on the context's stream for pw_estimate) without waiting for work the
 * caller has queued on other streams, so synchronise the producing stream first.  Host
 * memory is copied to the device on the lane's stream; pinned host memory (hipHostMalloc)
 * is read in place and asynchronously. */
typedef struct {
  const void *xyzw;
  const void *nbar;
  int64_t n;
  int dtype;
  int on_device;
} pw_catalog;

/* Normalisation scalars.  With use_given == 0 the library computes them (FP64 on the GPU)
 * and writes them back; with use_given == 1 it uses the caller's values. */
typedef struct {
  double alpha_r;
  double I;
  double S;
  int use_given;
} pw_norm;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device memory the
 * context may hold (0 = 90% of the device's free memory).  hip_stream (a hipStream_t, or
 * NULL) is the stream pw_estimate runs on; NULL makes the context create its own.
 * Tracing: with PW_TRACE=<file> in the environment when the context is created, every
 * completed estimate (pw_estimate, pw_estimate_orders, pw_estimate_batch, pw_estimate_noalloc
 * and served requests) appends one JSON line to <file>:
 *   {"t_ms": end, ms since pw_create; "kind": "estimate" | "orders" | "batch" | "noalloc" |
 *    "served"; "ticket": pw_submit's ticket (0 otherwise); "lane": 0 for pw_estimate-family
 *    calls, 1.. for serving lanes; "status": the request's code; "stat", "los", "n_mesh",
 *    "prec"; "n_gal", "n_ran"; "batch": catalogs in its launch; "queued_ms": submission to
 *    admission; "run_ms": admission (or the call) to completion, on the host's clock;
 *    "stages_ms": {stage: ms} from HIP events on the lane's stream, for launches of one
 *    catalog}.
 * Every lane then records stage events, which costs a few microseconds per estimate.  An
 * unwritable file fails pw_create with PW_EINVAL. */
int pw_create(pw_ctx **ctx, int device, size_t hbm_budget_bytes, void *hip_stream);

/* Release every device allocation, stream and host resource of the context.  Pending
 * submissions are cancelled first.  ctx may be NULL. */
int pw_destroy(pw_ctx *ctx);

/* Run one estimate synchronously.
 *   out      [n_ell][n_bins] multipoles (host, FP64), n_ell = ell_max/2 + 1
 *   bin_mean [n_bins] mean |k| (or |r|) of the modes in each bin (host, may be NULL)
 *   counts   [n_bins] modes (or grid separations) per bin (host, may be NULL)
 * Midpoint P_l with order > 0 requires the catalog extent on every axis to be at most
 * box_len / 2 (the convolution grows to twice the survey width, Section 3.2): PW_EINVAL.
 * xi_l requires the r-bins to end at or below box_len / 2 (separations beyond alias with
 * their periodic images): PW_EINVAL.
 * Built couplings: bisector xi_l for ell_max <= 6 and order <= 4; midpoint P_l for
 * ell_max <= 6 with order <= 4, and order 6 for ell_max <= 4 (PW_EINVAL otherwise); bisector
 * P_l and midpoint xi_l for every ell_max <= 8, order <= 8. */
int pw_estimate(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal,
                const pw_catalog *ran, pw_norm *norm, double *out, double *bin_mean,
                int64_t *counts);

/* n catalogs of one configuration at once (1 <= n <= 8): gal[i], ran[i] (and norm[i] when norm
 * is not NULL) describe catalog i; out holds [n][n_ell][n_bins], bin_mean and counts (may be
 * NULL) [n][n_bins].  For the bisector P_l (Section 5.2) with the default plan, each forward
 * pass and the contraction run once over every catalog's fields (a launch grid of fields x
 * catalogs; each catalog is painted into its own buffers), so n small meshes cost far fewer
 * launches than n estimates; other configurations run the catalogs one after another.  Each
 * catalog's result equals its pw_estimate result (to FP64 rounding of the shell sums).  Errors as
 * pw_estimate; every catalog's range and extent checks pass before any output is written.
 * The serving loop (pw_submit) batches pending requests the same way: requests of one such
 * configuration at n_mesh <= 256 that are pending together share one launch. */
int pw_estimate_batch(pw_ctx *ctx, const pw_config *cfg, int n, const pw_catalog *gal,
                      const pw_catalog *ran, pw_norm *norm, double *out, double *bin_mean,
                      int64_t *counts);

/* pw_estimate for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  It allocates no device memory and no
 * pinned host memory: every device buffer of the estimate (plan tables, mesh, spectrum buffers,
 * paint tiles, particle records) is carved from one static device array of 256 MiB that each
 * GPU the library runs on holds until the process ends; the results come back through a
 * pageable host buffer of the context.  Arguments, outputs and results are those of
 * pw_estimate, with two limits:
 *   - catalogs must be device-resident (on_device = 1): PW_EINVAL otherwise;
 *   - the estimate must fit the 256 MiB scratch (every estimator at 32^3, bisector P_l at
 *     64^3 with a few million particles): PW_ENOMEM with the bytes needed otherwise, before
 *     anything is written to the device.
 * Every call on a GPU uses that GPU's one scratch array, which keeps the last call's contents
 * (each call clears what it accumulates): calls that overlap on one GPU, from different
 * contexts or threads, race.  Plan tables are uploaded on every call (nothing is cached in the
 * scratch). */
int pw_estimate_noalloc(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal,
                        const pw_catalog *ran, pw_norm *norm, double *out, double *bin_mean,
                        int64_t *counts);

/* Contributions of each series order separately, for the same configuration and catalogs as
 * pw_estimate: slice o holds the terms of order theta^(2o) (parity-even midpoint alpha = 2o,
 * Sections 3.3 and 4.3; bisector beta = o, Sections 5.2 and 6), or for the all-parity midpoint
 * the terms of alpha = o (Sections 3.2 and 4.2).
 *   out      [n_orders][n_ell][n_bins] (host, FP64), n_orders = order/2 + 1 (all-parity
 *            midpoint: order + 1); the slices sum to pw_estimate's result.  The shot noise
 *            S / I belongs to slice 0 (the monopole has no term beyond zeroth order, so its
 *            higher slices vanish).
 *   bin_mean, counts, norm: as for pw_estimate.
 * Bisector P_l with a generated coupling (ell_max <= 6, order <= 4) runs one pass: one set of
 * forward transforms and a contraction that sends every order's terms to accumulators of their
 * own.  Every other configuration runs pw_estimate at orders 0, 2, .., order and returns the
 * differences of successive truncations.  Errors as pw_estimate; outputs written only on
 * success. */
int pw_estimate_orders(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal,
                       const pw_catalog *ran, pw_norm *norm, double *out, double *bin_mean,
                       int64_t *counts);

/* Correlation-function multipoles normalised by random pairs and corrected for the survey
 * window.  The paper divides xi_l by I and the bin volume and leaves the window alone; this
 * call adds the Landy-Szalay-style normalisation on top of the same estimator (cfg->stat must
 * be PW_XI, either line of sight and series form).  Per r-bin a:
 *   N_l(a)   the estimate's pair sum (pw_estimate's xi_l times I v_a);
 *   R_L(a)   the same sum for the randoms alone (w alpha_r n_r, with the data's normalisation;
 *            R_0 is the bin's weighted random-pair count), L = 0, 2, .., L_max;
 *   xi_rr    [n_ell][n_bins]  N_l / R_0;
 *   xi_edge  [n_ell][n_bins]  the solution of N_l / R_0 = sum_l' M_ll' xi_l',
 *            M_ll' = (2l+1) sum_L (l L l'; 0 0 0)^2 f_L (may be NULL);
 *   window   [L_max/2 + 1][n_bins]  f_L = R_L / R_0 (may be NULL).
 * L_max = 2 ell_max, capped at 8 (midpoint) or 6 (bisector, whose built couplings stop there);
 * *n_window receives L_max/2 + 1.  Bins without random pairs are 0.  Costs two estimates.
 * Errors as pw_estimate; outputs written only on success. */
int pw_estimate_xi_normalized(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal,
                              const pw_catalog *ran, pw_norm *norm, double *xi_rr, double *xi_edge,
                              double *window, int *n_window, double *bin_mean, int64_t *counts);

/* Serving.  pw_submit validates a request, enqueues it and returns a ticket at once (the
 * first request of a configuration on a context also builds its host plan on the calling
 * thread: tens of ms, about 0.3 s for a midpoint plan at 512^3); a
 * worker thread of the context admits pending requests in arrival order as soon as one of the
 * context's serving lanes is free and the request's device memory fits the HBM budget (the
 * workspaces, then the cached plans of idle lanes are evicted, least recently used first, to
 * make room).  A plan (tables only) stays resident on its lane for later requests of the same
 * configuration; all plans of a lane share one workspace (mesh and spectrum buffers) that
 * grows to the largest of them.  Host-side plans are cached per context.  Each lane
 * has its own HIP stream, so admitted requests of any size, mesh and estimator run
 * concurrently on the device.  The inputs and output buffers must stay valid until the ticket
 * completes or is cancelled; outputs are written when the request finishes.  Pageable host
 * catalogs are copied into pinned buffers the context owns (a pool of at most 8 GiB, reused
 * across requests) on the submitting thread, so that the lane's copy to the device runs
 * asynchronously beside other lanes' kernels; without room in the pool the request reads the
 * caller's memory when it is launched.
 *   pw_submit   PW_OK and *ticket, or an error for a malformed request / one that can never
 *               fit the budget (PW_ENOMEM), or PW_EBUSY while the context already holds its
 *               queue limit of requests pending or running; nothing is enqueued then.
 *   pw_poll     PW_EAGAIN while pending or running; otherwise the request's final status
 *               (PW_OK, PW_ECANCELED or the error of pw_estimate), after which the ticket is
 *               released (a later call on it returns PW_EINVAL).
 *   pw_wait     blocks until the request is final, returns and releases like pw_poll.
 *   pw_cancel   removes a request that has not been admitted (its status becomes
 *               PW_ECANCELED); PW_EBUSY if it is already running.
 * Submission functions may be called from one thread at a time; they may run concurrently
 * with pw_estimate calls on the same context. */
int pw_submit(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal,
              const pw_catalog *ran, pw_norm *norm, double *out, double *bin_mean,
              int64_t *counts, uint64_t *ticket);
int pw_poll(pw_ctx *ctx, uint64_t ticket);
int pw_wait(pw_ctx *ctx, uint64_t ticket);
int pw_cancel(pw_ctx *ctx, uint64_t ticket);
/* Number of serving lanes (1..8, default 2); only before the first pw_submit (PW_EBUSY
 * after). */
int pw_set_lanes(pw_ctx *ctx, int n_lanes);
/* Serving launches made so far and the requests they carried (a batched launch carries
 * several); either pointer may be NULL. */
int pw_serving_stats(pw_ctx *ctx, uint64_t *launches, uint64_t *requests);
/* Backpressure: pw_submit returns PW_EBUSY while max_in_flight requests of the context are
 * pending or running (1..2^30, default 1024; PW_EINVAL otherwise).  A lower limit applies to
 * later submissions only; requests already queued stay queued. */
int pw_set_queue_limit(pw_ctx *ctx, int64_t max_in_flight);

/* Copy an internal buffer of the context's most recent pw_estimate to host memory (for
 * per-stage checks).  what:
 *   0  painted node masses, [N][N][N] (z, y, x order; FP32 or FP64 by prec)
 *   1  bisector P_l: the z-pass output slots of the weighted fields, [nfields][nslots] complex
 *      (real-harmonic field index J*J + J + mu); every retained half-spectrum mode occupies
 *      exactly one slot
 *   2  bisector P_l: coordinate of each slot, [nslots] uint32 = kx | ky << 11 | kz << 22 (FFT
 *      indices; kx <= N/2), or 0xFFFFFFFF for a padding slot that holds no mode;
 *      PW_EINVAL for paths that keep full spectra
 * *needed receives the byte count; data are copied only when dst is not NULL and
 * dst_bytes >= *needed.  Synchronises the context's stream. */
int pw_inspect(pw_ctx *ctx, int what, void *dst, size_t dst_bytes, size_t *needed);

/* Stage timing.  With timing on, pw_estimate records a HIP event before each stage and after
 * the last one on the context's stream; pw_stage_info then reports, for stage index
 * 0 .. n-1 of the most recent estimate, its name, GPU time in milliseconds (-1 when timing
 * was off) and its algorithmic HBM bytes (the bytes the stage must read and write: inputs
 * once, outputs once).  pw_stage_info returns PW_EINVAL past the last stage. */
int pw_set_timing(pw_ctx *ctx, int on);
int pw_stage_info(pw_ctx *ctx, int stage, const char **name, double *ms, double *bytes);

/* Autotuning of the column passes (the forward y and z passes, the midpoint's fused z pass,
 * the inverse y pass).  Each has a few launch shapes (fields per workgroup, columns per
 * workgroup) that compute the same values at different speeds; candidate 0 is the default.
 * mode 1 (the default): the first launch of each shape key in the process times every
 * candidate twice on the estimate's own data (the estimate synchronises its stream once for
 * this) and keeps the fastest for the rest of the process; the environment variable
 * PW_TUNE=0 turns the timing off, and PW_TUNE_CACHE=<file> stores and reloads the choices.
 * mode 0: default shapes; mode 2 + i: candidate i wherever it exists (default elsewhere), for
 * tests and benchmarks.  PW_EINVAL for other modes. */
int pw_set_tuning(pw_ctx *ctx, int mode);
/* Entry `index` (0, 1, ..) of the process's tuning table: the shape key (NUL-terminated,
 * truncated to key_len), the chosen candidate, its time and the default's in milliseconds (-1
 * when loaded from PW_TUNE_CACHE).  Any output pointer may be NULL.  PW_EINVAL past the end. */
int pw_tune_entry(int index, char *key, size_t key_len, int *choice, double *ms_best, double *ms_default);

/* Message of the last error on this context ("" after a successful call), from any thread.
 * The returned string belongs to the calling thread and stays valid until that thread's next
 * pw_last_error call. */
const char *pw_last_error(const pw_ctx *ctx);

/* Device-memory footprint (bytes) pw_estimate needs for cfg with the given catalog sizes,
 * for host catalogs in the mesh precision with the randoms' nbar (device-resident catalogs
 * need less: no staging); host-only, needs no device. */
int pw_footprint(const pw_config *cfg, int64_t n_gal, int64_t n_ran, size_t *bytes);

/* Coupling tables used by the kernels, in the real spherical-harmonic basis
 *   y_l^0 = Y_l^0,  y_l^m = sqrt(2) (-1)^m Re Y_l^m,  y_l^-m = sqrt(2) (-1)^m Im Y_l^m  (m > 0),
 * for inspection and tests; host-only, needs no device.  kind:
 *   0  bisector: rows (l, nu, J1, mu1, J2, mu2, value) of the symmetrised real coupling
 *      S with sum_{beta <= order/2} B folded in (Appendix F), such that
 *      Re sum_m Y_l^{m*}(k^) sum B F[Y_J1^M d](-k) F[Y_J2^{m-M} d](k)
 *        = sum_nu y_l^nu(k^) sum_{(J1,mu1) <= (J2,mu2)} S Re(conj(R_J1mu1(k)) R_J2mu2(k)),
 *      R_Jmu = F[y_J^mu d].
 *   1  midpoint: rows (l, nu, J1, mu1, J2, mu2, value) for alpha = `alpha` (Phi, Appendix D):
 *      A_{l nu}(D) = sum Phi' y_J1^mu1(D^) |D|^alpha g_{alpha J2 mu2}(D).
 *   2  midpoint Legendre: rows (l, 0, J, 0, 0, 0, F^{alpha,l}_J) (Appendix E).
 *   3  midpoint all-parity: rows (l, nu, J1, mu1, J2, mu2, value) for alpha = `alpha`: phi
 *      (Appendix B) in the real basis with the (-1)^J2 of g folded in (Section 3.2):
 *      A_{l nu}(D) = sum phi' y_J1^mu1(D^) |D|^alpha IFT[conj(d) F[(2r)^-alpha y_J2^mu2 d]].
 *   4  midpoint all-parity Legendre: rows (l, 0, J, 0, 0, 0, f^{alpha,l}_J) (Appendix E).
 * Writes at most max_rows rows of 7 doubles to rows (may be NULL) and the row count to
 * n_rows. */
int pw_coupling_table(int kind, int ell_max, int order, int alpha, double *rows,
                      int64_t max_rows, int64_t *n_rows);

#ifdef __cplusplus
}
#endif
#endif /* PW_H */
