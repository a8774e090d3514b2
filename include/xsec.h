/* xsec.h - C ABI of libxsec.so: line-by-line opacity cross-sections on one MI355X.
 *
 * The operations follow the paper's statement of the method (arXiv 2510.20870, section
 * "Functionality of pyROX"): read a line list with its partition function and broadening
 * coefficients (bullet "Download and read files"), compute line strengths and widths at
 * the user's pressure and temperature (bullet "Compute line-strengths and -widths"), the
 * Voigt profile as the real part of the Faddeeva function (bullet "Compute line
 * profiles"), and sum the profiles into a cross-section per temperature-pressure point
 * (bullet "Combine and save") on any user grid (section "Similar tools").
 *
 * Physics conventions (the paper gives no formulas; these textbook forms are used):
 *   S (Einstein A form)  = g' A /(8 pi c nu0^2) exp(-c2 E''/T) (1 - exp(-c2 nu0/T)) / Q(T)
 *   S (reference form)   = S_ref Q(T_ref)/Q(T) exp(-c2 E''/T)/exp(-c2 E''/T_ref)
 *                            (1 - exp(-c2 nu0/T))/(1 - exp(-c2 nu0/T_ref))
 *   b_D (1/e half-width) = (nu0/c) sqrt(2 k_B T / m)
 *   gamma_L (HWHM)       = gamma_ref (P/P_ref) (T_ref/T)^n_T      (no natural width)
 *   V(d)                 = Re w((d + i gamma_L)/b_D) / (b_D sqrt(pi))
 *   sigma(nu_j)          = sum over lines with |nu_j - nu0_i| <= cut_i of S_i V_i
 * with the cut either fixed, or min(cap, mult * f_V) with f_V the Olivero-Longbothum
 * Voigt FWHM 0.5346 f_L + sqrt(0.2166 f_L^2 + f_G^2), f_L = 2 gamma_L,
 * f_G = 2 b_D sqrt(ln 2). The difference nu_j - nu0_i and the cut test are FP64.
 *
 * Units: wavenumber cm^-1, pressure bar, temperature K, mass amu, sigma cm^2/molecule.
 *
 * Conventions of every call:
 *   - returns an xs_status (0 = XS_OK, negative = error); no exception or abort crosses
 *     the ABI; xs_last_error() gives a message for the calling thread's last failure;
 *   - inputs are copied before the call returns; the caller keeps ownership of every
 *     pointer it passes; outputs are written into caller-owned memory;
 *   - handles become invalid after unload/free; a context is used from one thread at a
 *     time, except the serving calls (xs_submit .. xs_release), which are thread-safe.
 */
#ifndef XSEC_H
#define XSEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XS_ABI_VERSION 8

typedef enum {
  XS_OK = 0,
  XS_EINVAL = -1,      /* bad argument (null pointer, NaN, P <= 0, unknown enum, ...) */
  XS_ENOMEM = -2,      /* the request does not fit the context's HBM budget            */
  XS_EDEVICE = -3,     /* a HIP runtime call failed                                    */
  XS_ENOTFOUND = -4,   /* unknown handle                                               */
  XS_EUNSORTED = -5,   /* grid not strictly increasing                                 */
  XS_EBUSY = -6,       /* handle still referenced by pending requests                  */
  XS_ECANCELLED = -7,  /* request was cancelled                                        */
  XS_ETIMEOUT = -8     /* xs_wait timed out                                            */
} xs_status;

enum { XS_EINSTEIN_A = 0, XS_REF_STRENGTH = 1 };  /* strength form                   */
enum { XS_Q_POWER = 0, XS_Q_TABLE = 1 };          /* partition-function form         */
enum { XS_CUT_FIXED = 0, XS_CUT_MIN_FWHM = 1 };   /* line-wing cutoff rule           */
enum { XS_FP32_KAHAN = 0, XS_FP64 = 1 };          /* arithmetic of the profile sum   */
enum { XS_F64 = 0, XS_F32 = 1 };                  /* element type of sigma outputs   */

typedef struct xs_ctx xs_ctx;     /* opaque; one per device                              */
typedef uint64_t xs_lines_t;      /* resident line list                                  */
typedef uint64_t xs_grid_t;       /* resident wavenumber grid                            */
typedef uint64_t xs_req_t;        /* serving request                                     */
typedef struct xs_graph xs_graph; /* captured batched computation                        */

int xs_abi_version(void);

/* Create a context on HIP device `device` that may hold at most `hbm_budget_bytes` of
 * device memory (line lists + grids + scratch + request outputs); 0 = 90% of free
 * memory. *out receives the context. Errors: XS_EINVAL, XS_EDEVICE. */
int xs_create(int device, size_t hbm_budget_bytes, xs_ctx **out);
/* Free every resource of the context (waits for its device work). NULL is a no-op. */
void xs_destroy(xs_ctx *ctx);
/* Message of the calling thread's last failed call ("" if none). Never NULL. */
const char *xs_last_error(const xs_ctx *ctx);
/* Device facts: compute units, LDS bytes per workgroup, arch name ("gfx950"). */
int xs_device_info(xs_ctx *ctx, int *n_cu, size_t *lds_bytes, char *arch, size_t arch_len);
/* Bytes of device memory the context currently accounts against its budget. */
int xs_memory_used(xs_ctx *ctx, size_t *used, size_t *budget);

/* A line list as a host structure of arrays, n records (paper: "Download and read
 * files"). nu0 float64 [cm^-1]; A_or_Sref float32 (Einstein A [s^-1], or the strength at
 * T_ref [cm/molecule] for XS_REF_STRENGTH); E_low float32 [cm^-1]; gamma_ref float32
 * [cm^-1/bar] at T_ref; n_T float32; g_up uint16 (>= 1; unused by the reference form).
 * J_low uint16, the lower state's rotational quantum number, indexes the broadening
 * tables of the species (NULL: 0 for every line; unused without tables).
 * The arrays need not be sorted: the library keeps a stable sort by nu0 (ties keep the
 * input order). n = 0 is allowed (every sigma is then 0). */
typedef struct {
  size_t n;
  const double *nu0;
  const float *A_or_Sref;
  const float *E_low;
  const float *gamma_ref;
  const float *n_T;
  const uint16_t *g_up;
  const uint16_t *J_low;
} xs_lines_desc;

/* The species: strength form, molecular mass [amu], T_ref [K] (296 when 0),
 * P_ref [bar] (1 when 0), and Q(T) = q_a * T^q_b (XS_Q_POWER) or the linear
 * interpolation of the q_n nodes (q_T ascending, q_val) clamped at the ends
 * (XS_Q_TABLE; the table is copied).
 * Pressure broadening ("Compute line-strengths and -widths": several descriptions):
 * n_broad = 0 gives gamma_L = gamma_ref (P/P_ref) (T_ref/T)^n_T with each line's own
 * gamma_ref and n_T; n_broad > 0 broadening partners (at most 8) with volume mixing ratios
 * broad_vmr[b] >= 0 and tables over J of broad_nj entries (at most 4096),
 * gamma_L = (P/P_ref) sum_b broad_vmr[b] broad_gamma[b*nj + j] (T_ref/T)^broad_n[b*nj + j]
 * with j = min(J_low, nj - 1) (the tables are copied; gamma >= 0, all finite). */
typedef struct {
  int strength_form;
  double mass_amu;
  double T_ref;
  double P_ref;
  int q_kind;
  double q_a, q_b;
  const double *q_T;
  const double *q_val;
  size_t q_n;
  int n_broad;
  size_t broad_nj;
  const double *broad_vmr;
  const double *broad_gamma;
  const double *broad_n;
} xs_species_desc;

/* Copy a line list into HBM (26 bytes per line, sorted by nu0). Errors: XS_EINVAL
 * (NaN/negative fields, g_up = 0 with the Einstein form, bad species), XS_ENOMEM. */
int xs_load_lines(xs_ctx *ctx, const xs_lines_desc *lines, const xs_species_desc *species,
                  xs_lines_t *out);
/* Release a line list. XS_EBUSY while serving requests or graphs still reference it. */
int xs_unload_lines(xs_ctx *ctx, xs_lines_t lines);
/* Number of lines and resident bytes of a list. */
int xs_lines_info(xs_ctx *ctx, xs_lines_t lines, size_t *n, size_t *bytes);

/* Copy a wavenumber grid of n points into HBM. It must be finite and strictly increasing
 * (else XS_EUNSORTED); n >= 1. A wavelength grid is converted by the caller (or built
 * by xs_set_grid_wavelength for a fixed resolving power). */
int xs_set_grid(xs_ctx *ctx, const double *nu_cm1, size_t n, xs_grid_t *out);

/* Fixed resolving power ("Similar tools": any user grid, which lets the user fix
 * R = lambda / delta lambda): the wavelengths lambda_k = lambda_min (1 + 1/R)^k, k = 0, 1,
 * ... while lambda_k <= lambda_max (micrometres), as wavenumbers nu = 1e4 / lambda in
 * increasing order (so point j of a result is the wavelength lambda_(n-1-j)); a
 * cross-section per molecule is the same at a wavelength and at its wavenumber.
 * xs_wavelength_grid_host writes the n points into nu_out (host, capacity cap; with
 * nu_out NULL or cap too small only *n_out is set, XS_OK and XS_EINVAL respectively);
 * xs_set_grid_wavelength makes it a resident grid. XS_EINVAL for lambda_min <= 0,
 * lambda_max < lambda_min, R <= 0, non-finite values or more than 2^31 points. */
int xs_wavelength_grid_host(double lambda_min_um, double lambda_max_um, double R,
                            double *nu_out, size_t cap, size_t *n_out);
int xs_set_grid_wavelength(xs_ctx *ctx, double lambda_min_um, double lambda_max_um,
                           double R, xs_grid_t *out, size_t *n_out);
/* Release a grid. XS_EBUSY while serving requests or graphs still reference it. */
int xs_free_grid(xs_ctx *ctx, xs_grid_t grid);
/* Number of points of a resident grid. */
int xs_grid_info(xs_ctx *ctx, xs_grid_t grid, size_t *n);

typedef struct { double P_bar, T_K; } xs_pt;

/* Options of a computation. cut_cm1 is the fixed cut (XS_CUT_FIXED) or the cap of
 * min(cap, fwhm_mult * f_V) (XS_CUT_MIN_FWHM). Launch shape (each 0 = autotuned):
 * pts_per_lane (1, 2, 4 or 8) sets the grid tile of one wavefront to 64 * pts_per_lane
 * points; split (1..256) divides each tile's line window into that many independent work
 * items whose partial sums are added in a fixed order; waves_per_simd is the
 * occupancy the tile kernel is compiled for: 3..6 waves per SIMD, 2 the compiler's own
 * choice, 0 automatic (the tuned value, else 5 on the FP32 path with 1 or 2 points per
 * lane and the compiler's choice otherwise). The result does not depend on the launch
 * shape beyond FP32 rounding (bitwise for a fixed shape).
 * select_eps > 0 turns on main-contributor selection (named in "Functionality of pyROX"
 * as a way to speed up the profile computation; the paper does not define it): per tile of
 * the grid and (P, T) point, lines are dropped when the sum of their contributions' upper
 * bounds over the tile stays within select_eps times a lower bound of sigma over the tile,
 * so that sigma changes by at most select_eps * sigma at every point (plus the FP32
 * rounding and the error budget tol of the kept lines); 0 computes every line. Must be in
 * [0, 1).
 * out_dtype: the element type of sigma outputs, XS_F64 (float64) or XS_F32 (float32, the
 * FP64 sum rounded once to nearest); the arithmetic is the same for both.
 * tile_group: how the tiles of a workgroup share work. 1: each wavefront sums the far
 * lines of its own tile. 4: the four wavefronts of a workgroup take four neighbouring
 * tiles, and the lines far from the whole four-tile span, with that span inside their
 * cut, are expanded once about the span's centre, the expansion split among the four
 * wavefronts and added in a fixed order (FP32 path, fixed cut, no selection, 1 or 2
 * points per lane; XS_EINVAL otherwise). 0: automatic (4 where it applies and the cut
 * spans at least 3 kappa half-widths of a four-tile span at the grid's middle, kappa the far
 * threshold below, else 1).
 * tol: the error budget of the FP32 path's cheaper far forms, relative to each line's
 * contribution at each point (section "Functionality of pyROX" leaves the accuracy of the
 * profile to the implementation): 0 is the default budget 2e-7; otherwise tol must lie
 * in [2e-7, 1e-5] (XS_EINVAL). It sets where the shifted Lorentzian
 * (3/2 + 2 y^2) / r^4 <= tol, the doubly shifted Lorentzian 3/2 / r^4 <= tol and the
 * far-line polynomials |X| >= kappa H + 1.25 take over, kappa = 4.09 at the default and
 * 3.16 at 1e-5 (the polynomial's truncation within 0.65 tol, the rest for its FP32
 * recurrence); the other forms keep their own error (within 6e-7), and the FP32 sums add
 * theirs (below 1e-6). So sigma's relative error stays below tol + 2e-6. The FP64 path
 * ignores it. */
typedef struct {
  int cutoff_kind;
  double cut_cm1;
  double fwhm_mult;
  int precision;
  int pts_per_lane;
  int split;
  int waves_per_simd;
  double select_eps;
  int out_dtype;
  int tile_group;
  double tol;
} xs_opts;

/* sigma(nu_j; P_k, T_k) for k < npts on every point of `grid`, written to
 * sigma_out[k * n_grid + j] (row-major [npts][n_grid] of float64, or of float32 with
 * opts->out_dtype = XS_F32). With out_on_device != 0,
 * sigma_out is device memory, the work is enqueued on `stream` (a hipStream_t, NULL =
 * the null stream) and the call returns without waiting; otherwise sigma_out is host
 * memory and the call returns when it is filled. Each output element is produced by one
 * work item in a fixed line order, so repeated calls give bitwise identical results.
 * Errors: XS_EINVAL (P or T <= 0 or not finite, bad options), XS_ENOTFOUND, XS_ENOMEM,
 * XS_EDEVICE. */
int xs_compute(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts, size_t npts,
               const xs_opts *opts, void *sigma_out, int out_on_device, void *stream);

/* Allocation-free variant of xs_compute, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * It computes what xs_compute computes with the same kernels (bitwise the same result
 * for the same launch shape), into device memory sigma_dev (npts * n_grid elements of
 * opts->out_dtype), enqueued on `stream` (a hipStream_t, NULL = the null stream); it
 * returns without waiting and calls no allocation routine: the point table, the line
 * records and the split partials live in one static device array of
 * XS_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first context on that GPU
 * until the process ends, and the tiles are issued in ascending order. Limit: the point
 * table plus the records and partials of one batch of P-T points (32 bytes per line that
 * can reach the grid and per point, plus 8 bytes per grid point and split when the line
 * window of a tile is split) must fit that array, else XS_ENOMEM (larger tables are run
 * in several batches inside the call). Every call on one GPU, from any context or
 * thread, shares that GPU's array, and a call leaves its contents behind: calls whose
 * device work overlaps in time (different streams without ordering between them) race
 * and give wrong results; calls on one stream are ordered. Nothing in the array needs to
 * start at zero (each call writes what it reads). Errors as xs_compute. */
#define XS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int xs_compute_noalloc(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts,
                       size_t npts, const xs_opts *opts, void *sigma_dev, void *stream);

/* Number of (line, grid point) pairs inside the cutoff, per (P, T) point, counted on the
 * device with the same FP64 rule as xs_compute: counts_out[k] (host memory). With
 * opts->select_eps > 0 only the pairs of the lines that selection keeps count. */
int xs_count_evals(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts,
                   size_t npts, const xs_opts *opts, uint64_t *counts_out);

/* The same pairs split by the evaluation tier each point needs on the FP32 path (its own
 * x^2 + y^2 and y, the tiers of the Voigt approximation described with
 * xs_eval_series_host): tiers 0..4 are the far-region variants (shifted Lorentzian, then
 * the asymptotic series with 2, 3, 4, 6 terms), tiers 5..8 the FP64 core with 16, 20-24,
 * 32, 40 terms, tier 9 the FP32 small-y core. Core points with y < 0.1 count in tier 9 and
 * the others by y in tier 5 (y >= 1) or 6 (20 terms for y >= 0.3, 22 for y >= 0.1), so
 * tiers 7 and 8 stay empty; the kernels still take the FP64 core with 24 to 40 terms for
 * lines of y < 0.1 that share a sub-batch of 64 lines with a line of y >= 0.1. counts_out: npts * XS_N_EVAL_TIERS host values,
 * [k][tier]. Accounting only (the algorithmic work of a launch); the sum over tiers is
 * xs_count_evals. */
#define XS_N_EVAL_TIERS 10
int xs_count_evals_by_tier(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts,
                           size_t npts, const xs_opts *opts, uint64_t *counts_out);

/* Batched computation captured once in a hipGraph (its point table and scratch are owned
 * by the graph) and replayed by xs_graph_launch on any stream; sigma_dev is device memory
 * of npts * n_grid elements of opts->out_dtype. Every batch of P-T points the plan needs
 * (xs_compute's batching) is captured into the one graph. While a graph exists, its line
 * list and grid stay referenced: xs_unload_lines and xs_free_grid fail with XS_EBUSY.
 * xs_destroy releases the device resources of the context's remaining graphs; their
 * handles then only accept xs_graph_destroy (xs_graph_launch fails with XS_EINVAL). */
int xs_graph_create(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts,
                    size_t npts, const xs_opts *opts, void *sigma_dev, xs_graph **out);
int xs_graph_launch(xs_graph *g, void *stream);
void xs_graph_destroy(xs_graph *g);

/* ---------------------------------------------------------------------- serving
 * A request loop for cross-section requests (continuous batching). Requests wait in
 * arrival order until the serving arena (one device allocation, sub-allocated per
 * request) has room for their footprint; a request that does not fit yet may be passed
 * by later ones that fit, at most max_bypass times, after which admission waits for it.
 * An admitted request holds its block until it is done. Its work is cut into steps (the
 * parameter kernel of a batch of P-T points, tile-kernel launches over chunks of at
 * least step_items work items, the batch's reduction); a server thread keeps
 * max_inflight execution lanes (HIP streams) fed with steps, always taking the next step
 * of the admitted request with the least estimated remaining work, discounted by the
 * time it has waited (with two lanes or more, one lane only runs requests of a single
 * step). Requests that arrive while others run are thus admitted as memory frees up,
 * their kernels share the device with the others at step granularity, and short requests
 * do not wait behind long ones. A served request's result depends only on its own
 * inputs and options (the launch shape is planned from them alone), so it is bitwise the
 * same served alone or in any mix. With an automatic split (opts.split = 0) the server
 * plans shorter work items than xs_compute (at most 4096 lines each), so the two agree to
 * FP32 rounding; with the same explicit split they agree bitwise. Footprint = records (32 B per line that can
 * reach the grid and per P-T point of a batch) + split partials + the output when it
 * goes to host memory + the grid of a window request + the point table and tile order.
 * The lines (and grid) of a request stay referenced until it is done: unloading them
 * meanwhile fails with XS_EBUSY. */
typedef struct {
  int max_inflight;   /* execution lanes (HIP streams); 0 = 4                             */
  size_t mem_bytes;   /* serving arena; 0 = min(64 GiB, half of the free budget)         */
  int max_bypass;     /* times a waiting request may be passed; 0 = 8, < 0 = never      */
  int start_paused;   /* nonzero: queue requests but admit none until resumed            */
  int max_admitted;   /* requests admitted at once; 0 = 32                               */
  int step_items;     /* work items per tile-kernel step; 0 = 56 per CU (two rounds)     */
} xs_serve_opts;
/* Start the server (once per context; xs_submit starts one with defaults otherwise).
 * Errors: XS_EBUSY (already running), XS_ENOMEM (arena does not fit the budget). */
int xs_serve_start(xs_ctx *ctx, const xs_serve_opts *opts);
/* Stop or resume admissions (requests already running are not affected). */
int xs_serve_pause(xs_ctx *ctx, int paused);
/* Queue sigma(grid; pts) like xs_compute. sigma_out: host memory (filled when the request
 * is done) or, with out_on_device != 0, device memory written by the server's streams
 * (valid once the request is done). *out receives the request handle. Errors at submit:
 * XS_EINVAL, XS_ENOTFOUND, XS_ENOMEM (the footprint exceeds the whole arena). */
int xs_submit(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts, size_t npts,
              const xs_opts *opts, void *sigma_out, int out_on_device, xs_req_t *out);
/* The same for the uniform grid nu_j = nu_start + j * step, j < n_points, built on the
 * device inside the request's arena memory (no grid handle, no allocation). */
int xs_submit_window(xs_ctx *ctx, xs_lines_t lines, double nu_start, double step,
                     size_t n_points, const xs_pt *pts, size_t npts, const xs_opts *opts,
                     void *sigma_out, int out_on_device, xs_req_t *out);
/* *done = 1 once the request has finished (successfully, failed or cancelled). */
int xs_poll(xs_ctx *ctx, xs_req_t req, int *done);
/* Wait for the request (timeout_s < 0: no limit). Returns the request's final status
 * (XS_OK, XS_ECANCELLED, or the error it failed with, whose message xs_last_error then
 * gives), or XS_ETIMEOUT if it is still pending at the timeout. */
int xs_wait(xs_ctx *ctx, xs_req_t req, double timeout_s);
/* Cancel a request: a queued one finishes at once, an admitted one after the steps it has
 * in flight (its output is then incomplete); both end with XS_ECANCELLED. A finished
 * request is not affected. Returns XS_OK. */
int xs_cancel(xs_ctx *ctx, xs_req_t req);
/* Submit, admission and completion times in seconds on the monotonic clock
 * (CLOCK_MONOTONIC, the clock of std::chrono::steady_clock on Linux; a time not yet
 * reached is returned as -1). Submit is stamped on entry to xs_submit, completion when
 * the output is in sigma_out. */
int xs_request_times(xs_ctx *ctx, xs_req_t req, double *t_submit, double *t_admit,
                     double *t_done);
/* Forget a finished request (XS_EBUSY while it is pending). */
int xs_release(xs_ctx *ctx, xs_req_t req);
/* Admission rule on a simulated clock (host only, no device): n requests arriving at
 * arrive[i] (non-decreasing) that hold their arena block for duration[i] once admitted
 * and need footprint[i] bytes of an arena of mem_bytes, with at most max_admitted admitted
 * at once, admitted by the same policy and arena allocator as the server. Writes
 * admit_out[i], done_out[i] and the peak arena bytes in use. XS_ENOMEM if a footprint
 * exceeds the arena. */
int xs_sched_simulate(size_t n, const double *arrive, const double *duration,
                      const uint64_t *footprint, uint64_t mem_bytes, int max_admitted,
                      int max_bypass, double *admit_out, double *done_out,
                      uint64_t *peak_bytes);

/* ---------------------------------------------------------------------- autotuning
 * The launch shape has three parameters: points per lane (the tile of one wavefront is
 * 64 * pts_per_lane grid points), the work items per resident wavefront slot that the
 * automatic split aims at (which sets the line range of one item, i.e. how many 64-line
 * LDS chunks a wavefront walks per item), and the occupancy the tile kernel is compiled
 * for (waves_per_simd). xs_autotune times candidate shapes on probe blocks of the given
 * workload (up to three grid blocks, up to five of its P-T points evenly spaced over the
 * batch, every line that reaches them) and stores the fastest in a process-wide cache
 * under the workload's
 * class: device arch and CU count, precision, cutoff kind, the line density around the
 * grid middle (power of two of the lines within the cut) and the number of P-T points
 * (1, 2..16, more). Every later call with pts_per_lane, split and waves_per_simd all 0
 * uses the cached shape of its class (results then follow that shape, so they agree with
 * untuned runs to FP32 rounding, and bitwise among runs with the same cache). */
typedef struct {
  int pts_per_lane, split, waves_per_simd;  /* the tuned shape (waves_per_simd 2..6)    */
  int items_per_slot;                       /* the cached class parameter               */
  double probe_ms;                          /* probe time of the tuned shape            */
  double default_probe_ms;                  /* probe time of the untuned default        */
  int candidates;                           /* shapes timed                             */
  char key[192];                            /* the workload class                       */
} xs_tune_result;
int xs_autotune(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, const xs_pt *pts,
                size_t npts, const xs_opts *opts, xs_tune_result *out);
/* The class key of a workload (as xs_autotune stores it). */
int xs_tune_key(xs_ctx *ctx, xs_lines_t lines, xs_grid_t grid, size_t npts,
                const xs_opts *opts, char *key_out, size_t key_len);
/* The process-wide cache (host only): read/write one entry (waves_per_simd 2..6, as in
 * xs_opts), clear, and JSON persistence.
 * xs_tune_cache_load merges the file's entries (XS_ENOTFOUND: no such file, XS_EINVAL:
 * malformed); xs_tune_cache_save writes every entry. xs_tune_cache_get returns
 * XS_ENOTFOUND for a key not cached. */
int xs_tune_cache_put(const char *key, int pts_per_lane, int waves_per_simd,
                      int items_per_slot, double probe_ms);
int xs_tune_cache_get(const char *key, int *pts_per_lane, int *waves_per_simd,
                      int *items_per_slot, double *probe_ms);
int xs_tune_cache_clear(void);
int xs_tune_cache_size(size_t *n);
int xs_tune_cache_load(const char *path);
int xs_tune_cache_save(const char *path);

/* Kernel timing (measurement of the tile kernel, the Voigt evaluation and accumulation
 * step). With timing enabled, xs_compute and xs_count_evals record a HIP event pair on
 * the launch stream around every tile (or count) kernel launch; xs_kernel_time waits for
 * the recorded events, returns the summed duration in ms and the number of launches since
 * the previous call, and starts a new period. Graph capture records no events. Enabling
 * or disabling discards events not yet read. */
int xs_set_kernel_timing(xs_ctx *ctx, int enable);
int xs_kernel_time(xs_ctx *ctx, double *ms_sum, int *n_launches);

/* Collision-induced absorption ("Download and read files", "Combine and save": the paper
 * restructures CIA coefficients onto a wavelength- and temperature-dependent grid). The
 * database gives, per temperature, coefficients alpha at its own increasing wavenumbers:
 * n_blocks blocks, block k holding the nodes [offsets[k], offsets[k+1]) of nu_cm1 and
 * alpha (host arrays, offsets of n_blocks + 1 entries, offsets[0] = 0; nu strictly
 * increasing within a block). Every block is interpolated linearly in nu onto `grid`
 * (zero outside the block's range, its end nodes included):
 * out[k * n_grid + j] (host memory, float64, caller-owned). The temperatures are the
 * caller's bookkeeping. XS_EINVAL for bad offsets or non-finite / unsorted nodes. */
int xs_cia_regrid(xs_ctx *ctx, xs_grid_t grid, const size_t *offsets, size_t n_blocks,
                  const double *nu_cm1, const double *alpha, double *out);

/* Output regridding (section "Similar tools": results on any user wavelength or
 * wavenumber grid, which fixes the spectral resolution): n_rows cross-section rows computed
 * on resident grid `src` (at least 2 points), sigma_src[r * n_src + j] (float64), resampled
 * onto resident grid `dst` into out[r * n_dst + k] (float64), e.g. onto a fixed resolving
 * power grid from xs_set_grid_wavelength. Each row is read as the piecewise-linear
 * function through its grid nodes, zero outside [src_0, src_(n-1)].
 *   XS_REGRID_LINEAR:   that function at each destination point;
 *   XS_REGRID_BIN_MEAN: its mean over each destination point's bin: from the midpoint
 *     with the previous destination point to the midpoint with the next one (the first and
 *     last bins mirrored to the same half-widths; a single destination point takes the
 *     whole source range), clipped to the source range; 0 for a bin wholly outside it.
 *     The integral over a bin is exact for the piecewise-linear function, so bin means
 *     times bin widths add up to its integral over the bins' union.
 * With on_device != 0 both buffers are device memory and the work is enqueued on `stream`
 * (hipStream_t, NULL = the null stream); otherwise both are host memory and the call
 * returns when out is filled. Errors: XS_EINVAL (NULL, bad mode, n_rows outside
 * [1, 2^20], a source grid of one point), XS_ENOTFOUND, XS_ENOMEM, XS_EDEVICE. */
enum { XS_REGRID_LINEAR = 0, XS_REGRID_BIN_MEAN = 1 };
int xs_regrid(xs_ctx *ctx, xs_grid_t src, xs_grid_t dst, const double *sigma_src,
              size_t n_rows, int mode, double *out, int on_device, void *stream);

/* The Voigt function K(x, y) = Re w(x + iy) as the kernels evaluate it, for n host
 * points: on the device (xs_eval_voigt) or compiled for the host (xs_eval_voigt_host).
 * precision: XS_FP32_KAHAN (FP32 tiers: inside x^2 + y^2 < 49 the FP32 small-y core for
 * y < 0.1, else the FP64 core) or XS_FP64. */
int xs_eval_voigt(xs_ctx *ctx, const double *x, const double *y, size_t n, int precision,
                  double *K_out);
int xs_eval_voigt_host(const double *x, const double *y, size_t n, int precision,
                       double *K_out);

/* The far-region (x^2 + y^2 >= 49) FP32 forms of the tile kernel, compiled for the host,
 * for mapping their error (Voigt profile as Re w, section "Functionality of pyROX"): a line
 * lying outside a row of grid points is evaluated at every point of the row with the
 * variant its nearest point needs.
 *   variant 0: shifted Lorentzian (y / sqrt(pi)) / (x^2 + y^2 - 3/2);
 *   variant 1, 2, 3, 4: the asymptotic series of w with 2, 3, 4, 6 terms;
 *   variant -1: per point, the variant the kernel picks for a nearest point there under
 *   error budget `tol` (as xs_opts.tol: 0 the default 2e-7; the shifted Lorentzian where
 *   (3/2 + 2 y^2) / r^4 <= tol).
 * x, y, K_out: n host values; variant_out (NULL or n ints) receives the variant used.
 * Points with x^2 + y^2 < 49 or y <= 0, or an invalid tol, give XS_EINVAL. */
int xs_eval_series_host(const double *x, const double *y, size_t n, int variant, double tol,
                        double *K_out, int *variant_out);

/* The bounds of K(x, y) that main-contributor selection uses (FP32 arithmetic with
 * 1e-5 margins, compiled for the host, at x and y rounded to FP32):
 * K_lo = erf(2) (y / sqrt(pi)) / ((|x| + 2)^2 + y^2) <= K, and K <= K_hi = 1, or for
 * x^2 + y^2 >= 49 the shifted Lorentzian widened by twice its error bound. Either output
 * may be NULL; y must be > 0 (XS_EINVAL otherwise). */
int xs_eval_bounds_host(const double *x, const double *y, size_t n, double *K_lo,
                        double *K_hi);

/* The FP32 path's polynomial for far lines, compiled for the host (FP32 arithmetic at the
 * inputs rounded to FP32). A line whose doubly shifted Lorentzian K = (y / sqrt(pi)) /
 * (r^2 - 3/2 + 2 y^2 / r^2), r^2 = x^2 + y^2, holds over a whole tile (3/2 / r^4 <= eps at
 * its nearest point, any y: r^2 >= 2738.6 at the default budget), with every point of the
 * tile inside the cut, is summed as a polynomial of degree 13 in the tile coordinate
 * t in [-1, 1] when |X| >= kappa H + 1.25, X being x at the tile's centre and H the tile's
 * half-width in Doppler units; eps and kappa are those of budget `tol` (as xs_opts.tol: 0
 * the default, eps = 2e-7 and kappa = 4.09) (section
 * "Functionality of pyROX": the profile of every line inside the cutoff, here summed per
 * tile instead of per point). Where the shifted Lorentzian (y / sqrt(pi)) /
 * (x^2 + y^2 - 3/2) also holds at the nearest point, its expansion (truncation within
 * 1.3e-7 at the default budget) is taken, else the doubly shifted one's. K_out[i]: that
 * polynomial's K at x = X[i] + H[i] t[i]; kind_out (may be NULL): 0 for the shifted, 1 for
 * the doubly shifted expansion. Each case must meet the conditions above, have y > 0 and
 * |t| <= 1, and tol must be valid (XS_EINVAL otherwise). */
int xs_eval_far_host(const double *X, const double *H, const double *y, const double *t,
                     size_t n, double tol, double *K_out, int *kind_out);

#ifdef __cplusplus
}
#endif
#endif /* XSEC_H */
