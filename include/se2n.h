/*
 * se2n.h - C ABI of the MI355X (gfx950) library for the semi-discrete SE(2,N)
 * hypoelliptic diffusion of Boscain, Chertovskih, Gauthier and Remizov
 * ("Hypoelliptic diffusion and human vision: a semi-discrete new twist").
 *
 * The calls follow the paper's statement of the problem: an image f on an
 * M x M periodic grid with a set B of missing pixels is lifted to N discrete
 * orientations, diffused by the semi-discrete operator, and projected back to
 * the plane.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every data pointer is DEVICE memory owned by the caller, contiguous,
 *   row-major.  Images are [M][M] indexed [y][x] (x fastest); orientation
 *   volumes are [N][M][M] indexed [r][y][x].
 * - Real data (f, psi, out) has the plan's dtype: float for SE2N_F32, double
 *   for SE2N_F64.  Masks and orientation maps are uint8.
 * - mask[y][x] = 1 marks a missing pixel (the paper's bad set B), 0 a known one.
 * - Orientation r stands for the angle e_r = 2*pi*r/N.
 * - Every call only enqueues work on `stream` (a hipStream_t; NULL is the
 *   default stream) and returns; nothing is synchronised.  Device faults
 *   surface at the caller's next synchronisation.
 * - Every call returns SE2N_OK (0) or a negative se2n_status.  All argument
 *   checks happen on the host before anything is enqueued; a failed call
 *   enqueues nothing and leaves a message in se2n_last_error().  The library
 *   never aborts the process.
 * - A plan may be used from one host thread / one stream at a time.
 *
 * Time scale: the library integrates d psi/dt = D psi with D the totally
 * discrete operator of equation (FTE) (without its factor 1/2), i.e. per
 * spatial frequency A_{k,l} = beta*L - M*diag_r((a^r_{k,l})^2).  This is the
 * weighted operator Delta^(N) of Sec. "The weighting of the metric"; a time T_p
 * in the paper's (FTE) clock is T = T_p/2 here, and alpha = beta (2 pi/N)^2.
 */
#ifndef SE2N_H
#define SE2N_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SE2N_OK = 0,
    SE2N_EINVAL = -1,       /* bad argument: size, pointer, parameter range  */
    SE2N_EUNSUPPORTED = -2, /* valid for the paper, not supported by this build */
    SE2N_ENOMEM = -3,       /* device allocation of a library-owned buffer failed */
    SE2N_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
    SE2N_ESTATE = -5        /* plan destroyed or used inconsistently */
} se2n_status;

typedef enum { SE2N_F32 = 0, SE2N_F64 = 1 } se2n_dtype;

/* Time integration of each decoupled N x N system (proof of Theorem 2):
 * SE2N_CN    Crank-Nicolson with tau = T/n_steps (remark 2 after Theorem 2):
 *            psi(T) = R(tau A)^n psi(0), R(z) = (1 + z/2)/(1 - z/2);
 * SE2N_EXACT the exponential e^{T A} of equation (soleq). */
typedef enum { SE2N_CN = 0, SE2N_EXACT = 1 } se2n_scheme;

/* Projection to the plane (Sec. "A final inpainting algorithm ..."):
 * maximum over orientations (the paper's preferred choice) or the mean. */
typedef enum { SE2N_PROJ_MAX = 0, SE2N_PROJ_MEAN = 1 } se2n_proj;

typedef struct se2n_plan_s *se2n_plan;

/* Create a plan for M x M images and N orientations.
 * M: 16 <= M <= 4096, M = 2^a 3^b with a >= 2 (the FFTs are mixed radix 2/3;
 *    4 | M gives the frequency classes their (k, M/2 - k) pairing; sides
 *    with 8 !| M, e.g. 36, 108, 324, move 4 image rows at a time).
 * N: 4 <= N <= 64.  Even N lets each per-mode system split into two N/2
 *    blocks (the potential is pi-periodic, Sec. "The weighting of the
 *    metric", remark about projectivization): the fast path.  Odd N keeps
 *    one N x N propagator per frequency class (a plain solve kernel; the
 *    iterated schedule needs even N).
 * The plan owns twiddle tables (allocated here) and a cache of per-frequency
 * propagators (allocated on first use).  *out is set on success only.
 * Errors: SE2N_EINVAL (null out, bad M or N, bad dtype), SE2N_ENOMEM, SE2N_EHIP. */
int se2n_plan_create(se2n_plan *out, int M, int N, se2n_dtype dtype);

/* Free every buffer the plan owns.  Waits for the device first (hipDeviceSynchronize).
 * Passing NULL is SE2N_EINVAL. */
int se2n_plan_destroy(se2n_plan plan);

/* Bytes of device workspace that se2n_diffuse and se2n_inpaint need: the
 * half-spectrum volume [N][M/2+1][M] of complex values plus small scratch;
 * for FP32 plans of the sides with compiled passes (512, 1024, 2048) a
 * second volume of that size, into which the inverse column pass writes its
 * result in the row-blocked layout that the inverse row pass reads
 * contiguously.  Returns 0 for a NULL plan. */
size_t se2n_workspace_bytes(se2n_plan plan);

/* Solver schedule of the Crank-Nicolson diffusion (se2n_diffuse, se2n_inpaint;
 * SE2N_EXACT always uses the propagator):
 * SE2N_SCHEDULE_PROPAGATOR (default)  the n steps collapsed into one
 *     FP64-built propagator per frequency class (cached per (T, beta,
 *     n_steps)) and applied in one pass over the spectrum: cost independent
 *     of n once built; repeated calls give identical bits.
 * SE2N_SCHEDULE_ITERATED    the n steps taken one by one on every mode in
 *     registers (remark 2 after Theorem 2: Crank-Nicolson with a cyclic
 *     tridiagonal solver, Thomas + Sherman-Morrison; factors in FP64, steps in
 *     the plan's dtype): no precompute, cost proportional to n.
 * SE2N_SCHEDULE_AUTO  the cached table if there is one; for a key asked for
 *     the first time, the iterated steps when they are estimated cheaper
 *     than building the table; a key asked for again builds it (so the first
 *     and later results of a key differ by rounding). */
typedef enum {
    SE2N_SCHEDULE_AUTO = 0,
    SE2N_SCHEDULE_PROPAGATOR = 1,
    SE2N_SCHEDULE_ITERATED = 2
} se2n_schedule;
/* Errors: SE2N_EINVAL (unknown schedule), SE2N_EUNSUPPORTED (iterated with odd N). */
int se2n_set_schedule(se2n_plan plan, se2n_schedule schedule);
/* The schedule the plan's last diffusion ran (SE2N_SCHEDULE_AUTO before any).
 * Errors: SE2N_EINVAL (NULL), SE2N_ESTATE. */
int se2n_last_schedule(se2n_plan plan, se2n_schedule *schedule);

/* Fill the propagator cache for (T, beta, n_steps, scheme) now instead of on
 * the first diffusion (Remark 3 after Theorem 2: the matrices A_{k,l} are
 * universal once M, N and beta are fixed, so their propagators are computed
 * once).  The propagators are computed in FP64 on the device and stored in
 * the plan's dtype.
 * T >= 0, beta >= 0, n_steps >= 1 (ignored by SE2N_EXACT).
 * Errors: SE2N_EINVAL, SE2N_ENOMEM, SE2N_EHIP. */
int se2n_precompute(se2n_plan plan, double T, double beta, int n_steps,
                    se2n_scheme scheme, void *stream);

/* Frequency classes whose propagator is negligible for (T, beta, n_steps,
 * scheme): every entry below 2^-30 (FP32 plans) or 2^-60 (FP64 plans).  Their
 * modes are exactly zero at time T to within the rounding of the result
 * (the dropped part of a mode is at most (N/2) 2^-30 of its input), so the
 * diffusion takes them as zero: it reads neither the mode nor its propagator,
 * and for the sides with compiled column kernels (512, 1024, 2048 in FP32)
 * neither stores nor reloads the mode's spectrum lines when they hold no
 * live mode.
 * flags [Q][Q] uint8 host buffer, Q = M/4 + 1 (class (lx, ly) at lx*Q + ly):
 * 1 = negligible.  Computes the propagators on `stream` if they are not
 * cached, then waits for the stream.  *Q receives M/4 + 1; flags may be
 * NULL to query it, else capacity must be at least Q*Q.
 * Errors: SE2N_EINVAL (bad parameters, capacity too small), SE2N_ENOMEM, SE2N_EHIP. */
int se2n_propagator_flags(se2n_plan plan, double T, double beta, int n_steps,
                          se2n_scheme scheme, void *stream, uint8_t *flags, long capacity, int *Q);

/* Orientation map of the corrupted image (Sec. "A final inpainting algorithm
 * ...": Gaussian smoothing and gradient at the level of the FFT, nearest angle;
 * the gradient is taken on the corrupted image as the paper does).
 *   f      [M][M] real, mask [M][M] uint8 (1 = missing)
 *   sigma  Gaussian width in pixels, > 0, applied as the Fourier multiplier
 *          exp(-2 pi^2 sigma^2 (kbar^2 + lbar^2) / M^2)
 *   rmap   [M][M] uint8 out: r = floor(theta N/(2 pi) + 1/2) mod N with
 *          theta = atan2(g_y, g_x) + pi/2 the level-line direction of the
 *          smoothed central-difference gradient (g_x, g_y).
 *   workspace: at least se2n_workspace_bytes(plan) bytes.
 * Errors: SE2N_EINVAL (null pointer, sigma <= 0), SE2N_EHIP. */
int se2n_orient(se2n_plan plan, const void *f, const uint8_t *mask, double sigma,
                uint8_t *rmap, void *workspace, void *stream);

/* Which route se2n_orient (and se2n_inpaint without rmap_in) takes for sigma.
 * Both multipliers of the orientation step factor into an x part and a y
 * part, so the smoothed gradient is a separable circular convolution with
 * their inverse DFTs.  FP32 plans use that stencil when both kernels' tails
 * beyond some radius, or the whole circle, stay below 2^-26 of their
 * absolute sums and a compiled radius (8 .. 32) covers it: *radius receives
 * that compiled radius.  Otherwise (FP64 plans, wide or very narrow
 * Gaussians on large grids) the FFT route runs and *radius is 0.  The taps
 * are computed on the host in FP64, O(M^2) work, once per plan and sigma.
 * Errors: SE2N_EINVAL (null radius, sigma <= 0), SE2N_ESTATE. */
int se2n_orient_method(se2n_plan plan, double sigma, int *radius);

/* The stencil's taps themselves (host only, no device needed): for side M
 * (as se2n_plan_create) and sigma > 0, g[0..64] and d[0..64] receive the
 * correlation weights of offsets j = -32 .. 32 (index j + 32) of the
 * smoothing kernel and of the smoothed central difference, rounded to FP32,
 * zero beyond the radius; *radius receives the compiled radius, or 0 when
 * the stencil is not used at any precision (then g and d are untouched).
 * Errors: SE2N_EINVAL (bad M, sigma, null pointer). */
int se2n_orient_stencil_taps(int M, double sigma, float *g, float *d, int *radius);

/* Lift: psi[r][y][x] = f[y][x]*(1-mask[y][x]) if rmap[y][x] == r, else 0.
 *   psi [N][M][M] real out.  rmap values must be < N (not checked on device:
 *   a larger value lifts the pixel to no orientation).
 * Errors: SE2N_EINVAL, SE2N_EHIP. */
int se2n_lift(se2n_plan plan, const void *f, const uint8_t *mask, const uint8_t *rmap,
              void *psi, void *stream);

/* Diffuse an orientation volume in place to time T (Theorem 2: FFT over
 * (Z/MZ)^2 of every slice, the M^2 decoupled N-dimensional systems, inverse
 * FFT).  psi [N][M][M] real, in/out.  workspace: se2n_workspace_bytes bytes.
 * Parameters as in se2n_precompute; the propagators are taken from the cache
 * or computed (FP64) on the stream first.
 * Errors: SE2N_EINVAL, SE2N_ENOMEM, SE2N_EHIP. */
int se2n_diffuse(se2n_plan plan, void *psi, double T, double beta, int n_steps,
                 se2n_scheme scheme, void *workspace, void *stream);

/* Project a volume to the plane: out[y][x] = max_r psi[r][y][x] or the mean.
 * Errors: SE2N_EINVAL, SE2N_EHIP. */
int se2n_project(se2n_plan plan, const void *psi, se2n_proj mode, void *out, void *stream);

/* The whole path, fused so that the lifted volume never exists in real
 * space: orient -> lift + row FFT -> column FFT -> per-mode propagation ->
 * inverse column FFT -> inverse row FFT + projection.
 *   rmap_in  optional [M][M] uint8: if non-NULL it is used instead of
 *            computing the orientation map (values must be < N).
 *   rmap_out optional [M][M] uint8: receives the orientation map used.
 *   out      [M][M] real.
 * Errors: as se2n_orient and se2n_diffuse. */
int se2n_inpaint(se2n_plan plan, const void *f, const uint8_t *mask, double sigma,
                 double T, double beta, int n_steps, se2n_scheme scheme, se2n_proj mode,
                 const uint8_t *rmap_in, uint8_t *rmap_out, void *out, void *workspace,
                 void *stream);

/* ------------------------------------------------------------------------
 * Restoration heuristics (Sec. "Heuristic complements": subsections "Static
 * restoration (SR)" and "Dynamic restoration (DR)"; Appendix A, Table 1)
 * ------------------------------------------------------------------------
 * The pixels split into the good set G (known: mask = 0) and the bad set B.
 * [0, T] is cut into n_intervals intervals of tau = T / n_intervals with mesh
 * points t_i = i tau; each interval is integrated by `substeps` Crank-Nicolson
 * steps of tau / substeps (SE2N_CN) or by e^{tau A} (SE2N_EXACT).  At every
 * mesh point t_1 .. t_{n-1} the lifted state is mixed with its start on G:
 *     psi(x, y, theta) *= (eps h_ref + (1 - eps) h) / h,   h = max_theta psi,
 * at the pixels of G where h > 0 (elsewhere, including where h <= 0, where
 * the factor is undefined, psi is left unchanged); h_ref = h(x, y, 0) =
 * max(f, 0).  The state at T is projected without a final mix.
 * dynamic = 1 (DR): before each mix G grows by the bad pixels that have a
 * good 8-neighbour and whose h is larger than the mean of h over the bad
 * pixels of their 3x3 neighbourhood (themselves included; periodic grid;
 * all decisions of one mesh point taken from the sets before it).  A pixel
 * that joins at t_i has h_ref = h(x, y, t_i).
 * The paper's Table 1 gives alpha and T_p in its own clock: use
 * beta = alpha (N / 2 pi)^2 and T = T_p / 2 here (see the time scale above),
 * n_intervals = n, eps = epsilon.
 *   f, mask, sigma, rmap_in, rmap_out, mode, out: as se2n_inpaint.
 *   join_out optional [M][M] int16: the mesh index at which each pixel
 *            became good (0: known from the start, -1: never; SR: 0 or -1).
 *   workspace: se2n_restore_workspace_bytes(plan) bytes.
 * 0 <= eps <= 1, 1 <= n_intervals <= 32767, substeps >= 1, T >= 0, beta >= 0.
 * Errors: as se2n_inpaint; SE2N_EINVAL for the ranges above or dynamic not
 * 0 or 1. */
size_t se2n_restore_workspace_bytes(se2n_plan plan);
int se2n_restore(se2n_plan plan, const void *f, const uint8_t *mask, double sigma,
                 double T, double beta, int n_intervals, int substeps, se2n_scheme scheme,
                 double eps, int dynamic, se2n_proj mode, const uint8_t *rmap_in,
                 uint8_t *rmap_out, int16_t *join_out, void *out, void *workspace, void *stream);

/* se2n_inpaint without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and result as se2n_inpaint, but
 * instead of a caller workspace the call uses a static device array of
 * SE2N_NOALLOC_MAX_BYTES bytes inside the library (one per GPU, held until
 * the process ends).  It calls no hipMalloc, hipFree or other allocating
 * routine and creates no events (se2n_profile timing does not cover it).
 * Set-up, done before the first such call for a parameter set:
 *   - se2n_precompute(plan, T, beta, n_steps, scheme, ...) fills the
 *     propagator cache (this call never computes propagators), unless the
 *     plan's schedule is SE2N_SCHEDULE_ITERATED and the scheme SE2N_CN;
 *   - for an FP32 plan without rmap_in, se2n_orient_method(plan, sigma, ...)
 *     prepares the orientation stencil for sigma (host work).
 * The plan's device must be current.  Every call on one GPU shares that
 * GPU's array, and it keeps the last call's contents: calls that overlap in
 * time on one GPU (other streams, other plans, other threads) race and must
 * be ordered by the caller.  Nothing in the array needs to start at zero.
 * When the array is too small for the second (row-blocked) volume of
 * se2n_workspace_bytes, the inverse passes work in place on the first one
 * (same result, a slower inverse row pass).
 * Errors: as se2n_inpaint; SE2N_EINVAL if the workspace without that second
 * volume exceeds SE2N_NOALLOC_MAX_BYTES (e.g. M = 512 fits N <= 60, M = 1024
 * does not fit N = 16); SE2N_ESTATE if the propagators or the orientation
 * taps are not prepared, or another device is current; SE2N_EHIP. */
#define SE2N_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int se2n_inpaint_noalloc(se2n_plan plan, const void *f, const uint8_t *mask, double sigma,
                         double T, double beta, int n_steps, se2n_scheme scheme, se2n_proj mode,
                         const uint8_t *rmap_in, uint8_t *rmap_out, void *out, void *stream);

/* Kernel timing.  While enabled, every kernel the plan launches is bracketed
 * by two hipEvents recorded on the launch stream; se2n_profile_stats waits
 * for the recorded events and returns, per kernel name, the number of
 * launches and their summed duration.  Enabling (or disabling) clears the
 * statistics.  Timing adds two event records per launch; leave it off in
 * production.
 * se2n_profile_stats: out may be NULL to query the count only; at most
 * `capacity` entries are written; *count receives the number of kernels.
 * Errors: SE2N_EINVAL, SE2N_EHIP. */
typedef struct {
    char name[32];
    int launches;
    double total_ms;
} se2n_kernel_stat;

int se2n_profile(se2n_plan plan, int enable);
int se2n_profile_stats(se2n_plan plan, se2n_kernel_stat *out, int capacity, int *count);

/* ------------------------------------------------------------------------
 * Batched inpainting of many independent images (FP32)
 * ------------------------------------------------------------------------
 * The whole path of se2n_inpaint (orientation map computed, CN or EXACT,
 * max or mean projection) for `count` images of possibly different M, N,
 * T, beta, n_steps, sigma.  Each pass (orientation rows / columns /
 * inverse rows, lift + row FFT, column FFT, per-mode propagation, inverse
 * column FFT, inverse row FFT + projection) is ONE persistent launch over
 * the tiles of every image; the passes of a batch are captured once into a
 * hipGraph that each call replays with a single graph launch.
 *
 * The library keeps, per device and per batch signature (the list of
 * (M, N, n_steps, scheme, proj, T, beta, sigma) of the items, pointers
 * excluded), a batch plan: the FP64-precomputed propagator tables (one per
 * distinct (M, N, T, beta, n_steps, scheme)), twiddle tables, tile lists
 * and the instantiated graph.  The first call with a new signature builds
 * it (propagators computed on `stream`); later calls only upload the items'
 * pointers when they changed and launch the graph.  At most 4 signatures
 * are cached per device (least recently used dropped); se2n_batch_clear
 * frees them all.
 *
 * Items: M = 2^a 3^b, a >= 3, 16 <= M <= 1024; N even in [4, 64];
 * T >= 0, beta >= 0, sigma > 0, n_steps >= 1 for SE2N_CN; f, mask, out
 * non-NULL device pointers ([M][M] float / uint8 / float), rmap_out NULL or
 * [M][M] uint8 (receives the orientation map).  Outputs of different items
 * must not overlap.  count in [1, 4096].
 * Calls on one device that overlap in time must use different workspaces
 * and signatures or be ordered on one stream: a batch plan holds one
 * device-side item table. */
typedef struct {
    int M, N, n_steps;
    int scheme; /* se2n_scheme */
    int proj;   /* se2n_proj */
    int reserved;
    double T, beta, sigma;
    const float *f;
    const uint8_t *mask;
    uint8_t *rmap_out;
    float *out;
} se2n_item;

/* Schedule of a batch (what the autotuner chooses).
 *   wg_per_cu   persistent workgroups per compute unit for every pass
 *               (1..16); 0 launches one workgroup per tile instead.
 *   order       0: tiles of each pass sorted by decreasing cost (largest
 *               first), 1: image by image in item order.
 *   row_groups  slice groups of the lift and inverse row passes (1..64,
 *               clamped to N): >1 gives more, smaller tiles; the max
 *               projection then combines groups with integer atomics
 *               (extra clear and decode passes). */
typedef struct {
    int wg_per_cu;
    int order;
    int row_groups;
    int reserved;
} se2n_tune;

/* Device workspace bytes se2n_inpaint_batched needs for these items: per
 * item the half-spectrum volume (two for sides 512, 768 and 1024, whose inverse
 * passes go through a row-blocked copy), a max-combining buffer and an
 * orientation map.  Returns 0 if an item is invalid (see se2n_last_error). */
size_t se2n_batch_workspace_bytes(const se2n_item *items, int count);

/* Inpaint every item (see above).  workspace: at least
 * se2n_batch_workspace_bytes(items, count) bytes of device memory.
 * Errors: SE2N_EINVAL (count, item or pointer), SE2N_ENOMEM, SE2N_EHIP. */
int se2n_inpaint_batched(const se2n_item *items, int count, void *workspace, void *stream);

/* Autotuner: time the batch under each candidate schedule (wg_per_cu in
 * {0, 1, 2, 4} x order in {0, 1} x row_groups in {1, 2, 4}), `reps` graph
 * launches each after one warm-up, on `stream` (this call synchronises it),
 * and keep the fastest for this signature.  If table_path is non-NULL the
 * choice is also written there (one JSON object per line, keyed by the
 * device's architecture name and the signature hash; an existing entry for
 * the key is replaced).  best / best_ms may be NULL.  The items' outputs
 * hold the result of one of the runs (all candidates compute the same
 * result up to FP32 rounding order).
 * Errors: as se2n_inpaint_batched; SE2N_EINVAL if reps < 1; SE2N_EHIP if the
 * table file cannot be written. */
int se2n_batch_autotune(const se2n_item *items, int count, void *workspace, void *stream, int reps,
                        const char *table_path, se2n_tune *best, double *best_ms);

/* Read tuning entries written by se2n_batch_autotune; later batch plans
 * whose architecture and signature match use them.  The table named by the
 * environment variable SE2N_TUNE_TABLE, if set, is read at the first batched
 * call.  Lines that do not parse are skipped.
 * Errors: SE2N_EINVAL (NULL path), SE2N_EHIP (file cannot be read). */
int se2n_batch_load_tune_table(const char *path);

/* Set (tune non-NULL) or query the schedule used for this signature on the
 * current device; setting drops a cached plan of that signature so the next
 * call rebuilds it.  Precedence: se2n_batch_set_tune > loaded table >
 * defaults {wg_per_cu 2, order 0, row_groups 1}.  Host only.
 * Errors: SE2N_EINVAL (bad items, NULL out, tune field out of range). */
int se2n_batch_set_tune(const se2n_item *items, int count, const se2n_tune *tune);
int se2n_batch_get_tune(const se2n_item *items, int count, se2n_tune *out);

/* The tile list of one pass of a batch under `tune` (NULL: the current
 * schedule), in execution order, 4 ints per tile {item, a, b, c}:
 *   pass 0 orientation rows     {item, row block, 0, 1}
 *   pass 1 orientation columns  {item, first column kx, 0, 0}
 *   pass 2 orientation inverse  {item, row block, 0, 2}
 *          (passes 0-2 hold the items whose orientation takes the FFT
 *          route, see se2n_orient_method; pass 9 holds the others)
 *   pass 3 lift + row FFT       {item, row block, first slice, end slice}
 *   pass 4 forward column FFT   {item, first column, 0, 0}
 *   pass 5 per-mode propagation {item, lx, first ly, N}
 *   pass 6 inverse rows         {item, row block, first slice, end slice}
 *   pass 7 max clear / decode   {item, first pixel, pixel count, 0}
 *   pass 8 inverse column FFT on column pairs (k, M/2-k) with the pairing
 *          step of the real inverse row transform
 *                               {item, slice * blocks + pair block, 0, 0}
 *   pass 9 orientation stencil  {item, 128 x 32 tile (row-major), radius, 0}
 * tiles may be NULL to query *ntiles only; at most `capacity` tiles are
 * written.  Host only, no device work.
 * Errors: SE2N_EINVAL. */
int se2n_batch_tiles(const se2n_item *items, int count, const se2n_tune *tune, int pass, int *tiles,
                     int capacity, int *ntiles);

/* Per-pass timing of batched calls.  While enabled, se2n_inpaint_batched
 * launches the passes one by one (no graph) with hipEvents around each;
 * se2n_batch_profile_stats returns the launches and summed milliseconds per
 * pass name as se2n_profile_stats does.  Enabling or disabling clears them.
 * Errors: SE2N_EINVAL, SE2N_EHIP. */
int se2n_batch_profile(int enable);
int se2n_batch_profile_stats(se2n_kernel_stat *out, int capacity, int *count);

/* Free every cached batch plan on every device (waits for the device). */
int se2n_batch_clear(void);

/* Sizes of a plan: *M, *N, *dtype (any may be NULL).  Errors: SE2N_EINVAL, SE2N_ESTATE. */
int se2n_plan_info(se2n_plan plan, int *M, int *N, se2n_dtype *dtype);

/* ------------------------------------------------------------------------
 * Learned corrector (BF16 MFMA network; not from the paper)
 * ------------------------------------------------------------------------
 * A small residual network that maps the real-space volume psi[N][M][M]
 * diffused with n_coarse Crank-Nicolson steps towards the volume a finer
 * step count gives:  psi_out = psi + r(psi),  r = conv3(relu(conv2(relu(
 * conv1(psi))))), each conv a 3x3 cross-correlation with circular padding
 * (the grid is periodic, as the paper's discretisation), N -> 32 -> 32 -> N
 * channels.  Weights and activations are bfloat16, products accumulate in
 * FP32 (MFMA), parameters are kept in FP32 and trained with Adam by the
 * library's own forward and backward kernels.  The fine-step plain solve is
 * the reference the network is trained against and judged by.
 *
 * Parameter vector (27744 floats): for layers l = 1, 2, 3 the weights
 * W_l[o][c][tap] (32 x 32 x 9, tap = (dy+1)*3 + (dx+1) for the input offset
 * (dy, dx), output channel o, input channel c), then the biases b_l[o] (32).
 * Channels are padded to 32; weights reading input channels >= N (layer 1)
 * or writing output channels >= N (layer 3), and those biases, are held at
 * zero.  1 <= N <= 32; M must be a multiple of 16.
 * Volumes are FP32 device arrays [batch][N][M][M] (planar, as se2n_diffuse).
 * A network may be used from one host thread / one stream at a time. */
typedef struct se2n_cnn_s *se2n_cnn;

/* Create a network with seeded He-normal weights in layers 1 and 2 and zero
 * layer 3 (it starts as the identity map); Adam state zero.
 * Errors: SE2N_EINVAL (null out, N out of range), SE2N_ENOMEM, SE2N_EHIP. */
int se2n_cnn_create(se2n_cnn *out, int N, uint64_t seed);
/* Waits for the device, frees the network.  Errors: SE2N_EINVAL. */
int se2n_cnn_destroy(se2n_cnn cnn);
/* Copy the FP32 parameters to host memory (synchronises the device).
 * host may be NULL to query *count (27744).  Errors: SE2N_EINVAL (capacity). */
int se2n_cnn_get_params(se2n_cnn cnn, float *host, int capacity, int *count);
/* Replace the parameters from host memory (padded entries forced to zero)
 * and reset the Adam state.  Errors: SE2N_EINVAL (count, non-finite). */
int se2n_cnn_set_params(se2n_cnn cnn, const float *host, int count);
/* The Adam optimiser's state (first and second moments, 27744 floats each,
 * and the step counter), for checkpointing and resuming training:
 * se2n_cnn_get_adam copies it to host memory (m and v may both be NULL to
 * query *step only; synchronises the device); se2n_cnn_set_adam replaces it
 * (call after se2n_cnn_set_params, which resets it).  Errors: SE2N_EINVAL
 * (NULL, count or capacity, non-finite values, v < 0, step < 0), SE2N_EHIP. */
int se2n_cnn_get_adam(se2n_cnn cnn, float *m, float *v, int capacity, int *step);
int se2n_cnn_set_adam(se2n_cnn cnn, const float *m, const float *v, int count, int step);
/* Workspace bytes of se2n_cnn_forward (training = 0) or of the gradient and
 * training calls (training = 1) for `batch` volumes of side M; 0 if invalid. */
size_t se2n_cnn_workspace_bytes(se2n_cnn cnn, int M, int batch, int training);
/* out = psi + r(psi) for `batch` volumes; out may equal psi.
 * Errors: SE2N_EINVAL (M not a multiple of 16, null pointer), SE2N_EHIP. */
int se2n_cnn_forward(se2n_cnn cnn, const float *psi, float *out, int M, int batch, void *workspace,
                     void *stream);
/* Gradient of the mean squared error between psi_coarse + r(psi_coarse) and
 * psi_fine over all batch*N*M*M values, with respect to the parameter
 * vector: grads (device, 27744 floats) and, if loss is non-NULL, the loss
 * (device, one float).  Every sum runs in a fixed order (deterministic). */
int se2n_cnn_gradients(se2n_cnn cnn, const float *psi_coarse, const float *psi_fine, int M, int batch,
                       float *grads, float *loss, void *workspace, void *stream);
/* One Adam step (bias-corrected, step counter kept by the network) with the
 * given device gradient.  Errors: SE2N_EINVAL (lr < 0, betas outside [0, 1),
 * eps <= 0). */
int se2n_cnn_adam_step(se2n_cnn cnn, const float *grads, float lr, float beta1, float beta2, float eps,
                       void *stream);
/* se2n_cnn_gradients + se2n_cnn_adam_step (beta1 0.9, beta2 0.999, eps 1e-8);
 * loss (device float) may be NULL. */
int se2n_cnn_train_step(se2n_cnn cnn, const float *psi_coarse, const float *psi_fine, int M, int batch, float lr,
                        float *loss, void *workspace, void *stream);
/* Per-kernel timing of the network's launches, as se2n_profile / se2n_profile_stats. */
int se2n_cnn_profile(se2n_cnn cnn, int enable);
int se2n_cnn_profile_stats(se2n_cnn cnn, se2n_kernel_stat *out, int capacity, int *count);

/* Record the measured accuracy of the network in one regime: applied to the
 * volume after n_coarse steps (scheme) to time T at side M with weight beta,
 * its volume rel-L2 against the n_fine-step FP64 solve was rel_l2.  A record
 * with the same key is replaced.  The records are the network's licence for
 * se2n_inpaint_corrected (below); se2n_cnn_get_validation returns a record's
 * rel_l2, or -1 if there is none.  Host only.
 * Errors: SE2N_EINVAL (sizes, non-finite parameters, rel_l2 < 0, NULL). */
int se2n_cnn_set_validation(se2n_cnn cnn, int M, double T, double beta, int n_coarse, int n_fine,
                            se2n_scheme scheme, double rel_l2);
int se2n_cnn_get_validation(se2n_cnn cnn, int M, double T, double beta, int n_coarse, int n_fine,
                            se2n_scheme scheme, double *rel_l2);

/* Workspace bytes of se2n_inpaint_corrected (0 if the plan is not FP32, N
 * differs from the network's, or M is not a multiple of 16). */
size_t se2n_corrected_workspace_bytes(se2n_plan plan, se2n_cnn cnn);
/* Inpainting with the corrector, with the fine-step plain solve as fallback
 * and judge.  If the network holds a validation record for (M, T, beta,
 * n_steps, n_fine, scheme) whose rel_l2 is at most max_rel_l2: orient, lift
 * to a real-space volume (in the workspace), diffuse with n_steps coarse
 * steps, psi += r(psi), project.  Otherwise the result cannot be shown to
 * meet the bar and the call runs the plain fused path (se2n_inpaint) with
 * n_fine steps instead.  *used_fallback (host int, may be NULL) receives 1
 * when the fallback ran, else 0.  rmap_out and out are [M][M] device arrays
 * (uint8, float).
 * Errors: as se2n_inpaint; SE2N_EINVAL if n_fine < n_steps or max_rel_l2 < 0;
 * SE2N_EUNSUPPORTED for FP64 plans. */
int se2n_inpaint_corrected(se2n_plan plan, se2n_cnn cnn, const void *f, const uint8_t *mask, double sigma,
                           double T, double beta, int n_steps, int n_fine, se2n_scheme scheme,
                           se2n_proj mode, double max_rel_l2, uint8_t *rmap_out, void *out,
                           int *used_fallback, void *workspace, void *stream);

/* Test hook for the error paths: after `after` more successful device (or
 * pinned host) allocations by the library, every later one fails as if the
 * memory were exhausted, until the hook is reset with after = -1 (the
 * default).  Calls that then need memory return SE2N_ENOMEM and free what
 * they had allocated.  Process-wide.  Errors: SE2N_EINVAL (after < -1). */
int se2n_debug_fail_allocations(long after);

/* Message describing the last failure on the calling thread ("" if none). */
const char *se2n_last_error(void);

/* Library version string. */
const char *se2n_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SE2N_H */
