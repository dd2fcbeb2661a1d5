/*
 * pngf.h -- C ABI of libpngf: the per-iteration hot path of the Precomputed
 * Numerical Green Function (PNGF) method for pixel inverse design, for one
 * AMD MI355X (gfx950).
 *
 * Problem statement (Results: Precomputation; Direct binary search;
 * Low-rank update evaluation; Supplementary Note 4, generalized materials):
 * a static 2D TM (Ez) FDFD environment is folded once into a dense design-
 * region Green function G (N_d x N_d), the background field b on the design
 * region and an output projection G_OD (1 x N_d) with background output x_b.
 * A design with permittivity contrast deps (per pixel, 0 or eps_hi-eps_lo) is
 * then solved exactly on the design region only:
 *
 *     (I - k0^2 G diag(deps)) E = b,      x = x_b + k0^2 G_OD diag(deps) E,
 *
 * and direct binary search flips one pixel at a time, keeping C^-1 current
 * with Sherman-Morrison updates (the rank-1 case, M = 1, of the paper's
 * Woodbury update, eq. lru_woodbury) and scoring candidate flips from the
 * current inverse without forming the new one (eq. lru_eobj_rs, here in field
 * form).  The objective, to be maximized, is f = mean_f |x_f|^2 / norm_f.
 *
 * Perfectly conducting pixels (pixel_kind PNGF_PIXEL_PEC; the paper's own
 * devices, eq. currequiv_j_disc): with P = diag(bits) the paper solves
 * [(I - P) + P G] j = P e_inc.  Its transpose is a field-form matrix,
 *
 *     (I - P + P G)^T = I - kappa (G - I) P   with kappa = -1,
 *
 * and z = (I - kappa (G - I) P)^-1 b holds the total field on open pixels
 * and the paper's equivalent current j on conducting ones (field there is
 * zero; on the design region the field is b - G j), with
 * x = x_b + kappa G_OD P z.  So a PEC problem runs on the same kernels with
 * G - I in place of G and kappa = -1 in place of k0^2 deps at every
 * frequency; the paper's rank-M update (eq. lru_dcn, U = Q^T H_P,
 * V = Q (G - I)) is the transpose of the column update applied here.
 *
 * Conventions
 *   - All calls return int: 0 on success, a negative pngf_status otherwise;
 *     pngf_last_error(h) (or pngf_last_error(NULL) for a failed create) gives
 *     a message.  No call aborts the process.
 *   - Complex arrays are interleaved (re, im) doubles: "cplx[n]" means 2n
 *     doubles.
 *   - Every host array passed in is copied; the caller keeps ownership.
 *   - Device memory is caller-supplied (pngf_bind): the library never
 *     allocates device memory.  All device work is ordered on the bound HIP
 *     stream; calls that return host results synchronize that stream.
 *   - 2D arrays are (ny, nx) row-major, node n = j*nx + i.  Design pixels are
 *     numbered in that order restricted to the design mask.
 *   - A handle is not thread-safe; use one handle per thread.
 */
#ifndef PNGF_H
#define PNGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pngf_status {
  PNGF_OK = 0,
  PNGF_EINVAL = -1,     /* bad sizes, mask in the PML, pixel out of range  */
  PNGF_ESINGULAR = -2,  /* zero pivot in a factorization                   */
  PNGF_ENUMERIC = -3,   /* NaN/Inf or drift that a refresh cannot repair   */
  PNGF_EDEVICE = -4,    /* HIP runtime error                               */
  PNGF_ESTATE = -5,     /* call out of order (e.g. not bound, no design)   */
  PNGF_ENOMEM = -6      /* host allocation failed / workspace too small    */
} pngf_status;

enum { PNGF_POINT_INTENSITY = 0, PNGF_OVERLAP_INTENSITY = 1,
       PNGF_MEAN_TRANSMISSION = 2 };

/* pngf_problem.pixel_kind: a design bit selects eps_hi over eps_lo
 * (dielectric), or a perfect conductor (Ez = 0 on the pixel's node) over
 * eps_lo (PEC; eps_hi is then unused). */
enum { PNGF_PIXEL_DIELECTRIC = 0, PNGF_PIXEL_PEC = 1 };

/* PNGF_FP64_PLAIN: FP64 C^-1 kept current by a Sherman-Morrison update per
 *   accept (eq. lru_woodbury, M = 1); every candidate scored from C^-1 and G.
 * PNGF_MIXED: complex-FP32 C0^-1 with a deferred panel, FP64 refreshes and
 *   FP64 decisions inside the FP32 error band.
 * PNGF_RFORM: FP64 reduced scoring, not in the paper.  By reciprocity
 *   T = C^-1 G is complex symmetric, so an accept of pixel m changes it by
 *   alpha p p^T with p = T[:, m]; from T0 = C^-1 G at the run start and a
 *   panel of the p vectors, every candidate is scored from diag(T), E, R' in
 *   O(1) and an accept costs O(N_d k) instead of O(N_d^2).  Exact (same
 *   accepted sequence as the other forms).  Only pngf_dbs_run uses the
 *   R-form; the other calls bring C^-1 up to date first. */
enum { PNGF_FP64_PLAIN = 0, PNGF_MIXED = 1, PNGF_RFORM = 2 };

/* pngf_options.flags: record HIP events around every hot-path kernel launch
 * so pngf_kernel_times can report average device time per kernel. */
#define PNGF_FLAG_TIMING 1ull
/* pngf_options.flags: run every step of the mixed search as its own kernel
 * launch.  Without it, a single-frequency mixed search with N_d <= 2048 runs
 * each batch of steps as one launch whose workgroups (N_d / 8, at most one
 * per compute unit) keep their rows of C0^-1 in registers and meet at a grid
 * barrier between steps (same arithmetic, same results); it falls back to
 * one launch per step by itself where the grid cannot be resident at once.
 * Its barrier waits are bounded: if the device is shared and the workgroups
 * cannot all run, the search fails with PNGF_ENUMERIC after about a second
 * instead of waiting for ever. */
#define PNGF_FLAG_STEP_LAUNCHES 2ull
/* pngf_options.flags: like PNGF_FLAG_TIMING, but only the launches of search
 * steps (kernel class "accept") are timed, which keeps the events' own cost
 * off every other launch. */
#define PNGF_FLAG_TIMING_STEPS 4ull
/* pngf_options.flags: invert the FP64 system matrix with the pivot search
 * every time.  Without it, the S block of C (the pixels at eps_hi) is first
 * inverted by blocked Gauss-Jordan on 64-column panels without row
 * exchanges, whose rank-64 updates run on the FP64 matrix cores; a zero pivot
 * of a diagonal block, or a probe residual ||K K^-1 v - v||_inf above
 * tol (||K||_inf ||K^-1 v||_inf + ||v||_inf) for a fixed v (tol from
 * pngf_set_inverse_check), sends that inversion to the pivot search
 * instead.  Either way the result is C^-1 in FP64. */
#define PNGF_FLAG_PIVOT_SEARCH 8ull

typedef struct pngf_handle pngf_handle;

/* Input problem: the static environment, design region, sources, output
 * functional and frequencies (Results, Precomputation).  Units: lengths in
 * lambda0, c0 = eps0 = mu0 = 1, k0 = 2 pi f / f0. */
typedef struct pngf_problem {
  int32_t nx, ny, npml;        /* Ez nodes per axis; PML cells per side      */
  double h;                    /* grid step (units of lambda0)               */
  const double *eps_static;    /* [ny*nx] real relative permittivity; design */
                               /* cells must hold eps_lo                     */
  const uint8_t *design_mask;  /* [ny*nx] 1 = design pixel; must keep one    */
                               /* cell away from the PML and the grid edge   */
  double eps_lo, eps_hi;       /* binary pixel levels                        */
  int32_t nfreq;               /* number of frequencies (>= 1)               */
  const double *k0;            /* [nfreq]                                    */
  const double *src;           /* cplx[nfreq*ny*nx] current density J        */
                               /* (right-hand side i k0 J)                   */
  int32_t nobj;                /* must be 1                                  */
  const double *w;             /* cplx[ny*nx] output functional, x = w^T E   */
  int32_t objective_kind;      /* PNGF_*_INTENSITY / MEAN_TRANSMISSION       */
  const double *obj_norm;      /* [nfreq] normalizers, or NULL for all 1     */
  int32_t pixel_kind;          /* PNGF_PIXEL_DIELECTRIC or PNGF_PIXEL_PEC    */
} pngf_problem;

typedef struct pngf_options {
  int32_t precision;    /* PNGF_FP64_PLAIN or PNGF_MIXED                     */
  int32_t k_refresh;    /* MIXED: FP64 refresh every k_refresh accepts;      */
                        /* 0 = only when the FP64 residual of E drifts.  A   */
                        /* refresh is a block-Woodbury update of the FP64    */
                        /* inverse of the last refresh (exact to rounding),  */
                        /* or a full re-inversion if > 64 pixels changed.    */
                        /* RFORM: every min(k_refresh, 64) accepts C^-1 is   */
                        /* re-inverted in FP64 and T0, E, R', x re-formed    */
                        /* from it, which bounds the growth of rounding in   */
                        /* the incremental updates; 0 = never                */
  int32_t k_fold;       /* MIXED: fold the deferred panel into C0^-1 once it */
                        /* holds k_fold terms (0 = only when it is full);    */
                        /* RFORM: panel capacity before a fold into T0       */
                        /* (0 = 512)                                         */
  int32_t max_accepts;  /* capacity of the on-device accept log (>= 1)       */
  int32_t max_sweeps;   /* largest n_sweeps pngf_dbs_run will be given       */
  int32_t max_tile;     /* PLAIN: largest tile (pixels flipped together,     */
                        /* <= 64) pngf_tile_dbs_run will be given; 0 = none  */
  double eta;           /* accept iff f' - f > eta * f (1e-9)                */
  double guard;         /* MIXED: relative FP32 error band of a score; a     */
                        /* candidate inside it is decided on the FP64 state; */
                        /* 0 = calibrated at every FP64 re-inversion         */
  uint64_t flags;       /* PNGF_FLAG_* bits                                  */
} pngf_options;

/* Result summary of a DBS run. */
typedef struct pngf_dbs_result {
  int32_t n_accepted;   /* accepted flips                                    */
  int32_t sweeps;       /* sweeps started                                    */
  int32_t converged;    /* 1 if a whole sweep had no improving flip          */
  int32_t n_refresh;    /* FP64 refreshes performed (MIXED)                  */
  int64_t attempts;     /* attempted flips (visited positions)               */
  int64_t n_verified;   /* MIXED: candidates re-checked in FP64              */
  double f_initial;     /* objective of the initial design                   */
  double f_final;       /* objective of the final design (FP64)              */
} pngf_dbs_result;

const char *pngf_version(void);
const char *pngf_last_error(const pngf_handle *h);

/* Precompute (host, FP64, OpenMP; timed separately).  Assembles the
 * symmetric FDFD operator with SC-PML and the source / output columns,
 * eliminates everything outside the design region by a nested-dissection
 * multifrontal Schur complement (the idea of the paper's augmented partial
 * factorization, Results, Precomputation), and inverts the design-region
 * Schur complement by nested-dissection-ordered block sweeps, giving per
 * frequency G = -(L^-1)[D,D] (exactly symmetric), b, G_OD and x_b.  G, b,
 * G_OD and x_b depend only on the environment, so they are the same for both
 * pixel kinds.  Frequencies run concurrently.  With objective_kind
 * PNGF_MEAN_TRANSMISSION each frequency's normalizer is obj_norm[f] (or 1)
 * times the vacuum transmission |w^T E_vac|^2 of the same source (eps = 1 on
 * the whole grid), from one more elimination.
 * Errors: PNGF_EINVAL for inconsistent sizes, a mask touching the PML or an
 * unknown pixel_kind / objective_kind, PNGF_ESINGULAR for a singular pivot
 * block, PNGF_ENUMERIC for a zero vacuum transmission, PNGF_ENOMEM. */
int pngf_precompute(const pngf_problem *p, pngf_handle **out);

/* Copies of the precomputed quantities of frequency fi (host arrays supplied
 * by the caller; any pointer may be NULL): G cplx[n_d*n_d] row-major,
 * b cplx[n_d], god cplx[n_d], xb cplx[1]. */
int pngf_get_precompute(pngf_handle *h, int32_t fi, double *G, double *b,
                        double *god, double *xb);

/* Objective normalizer norm_f of frequency fi (the objective is the mean
 * over frequencies of |x_f|^2 / norm_f): obj_norm[fi] (or 1), times the
 * vacuum transmission for PNGF_MEAN_TRANSMISSION.  Errors: PNGF_EINVAL for a
 * NULL handle / pointer or fi out of range. */
int pngf_objective_norm(pngf_handle *h, int32_t fi, double *norm);

/* Number of design pixels / frequencies of the handle. */
int pngf_sizes(pngf_handle *h, int32_t *n_d, int32_t *nfreq);

/* Host seconds spent in pngf_precompute. */
int pngf_precompute_seconds(pngf_handle *h, double *seconds);

/* Device bytes pngf_bind needs for these options. */
int pngf_workspace_bytes(pngf_handle *h, const pngf_options *o, size_t *bytes);

/* Bind caller-owned device memory (>= pngf_workspace_bytes, 256-byte aligned)
 * and a hipStream_t (NULL = default stream); uploads G, b, G_OD, x_b.
 * PNGF_ENOMEM if bytes is too small.  Memory of an earlier binding may still
 * be written by an initial inverse that pngf_set_design queued: this call
 * (and pngf_destroy) first waits for it, so the caller releases that memory
 * only after either returns. */
int pngf_bind(pngf_handle *h, const pngf_options *o, void *dev_ws, size_t bytes,
              void *hip_stream);

/* Set the design (bits[n_d], 0/1) and form the initial inverse
 * C0^-1 = (I - k0^2 G diag(deps))^-1 (its PEC counterpart above), E = C0^-1 b,
 * the output row
 * R' = G_OD (I + k0^2 diag(deps) C0^-1 G) and x (Direct binary search: the
 * inverse of the initial system matrix is found and stored).  FP64 on the
 * GPU: blocked Gauss-Jordan without row exchanges, checked by a probe
 * residual, and with the pivot search where that check fails.  Returns once
 * the inversion is queued: the check runs when the handle is next used (any
 * call below that needs a design, pngf_inverse_stats, pngf_kernel_times),
 * which then reports PNGF_ESINGULAR for a zero pivot and drops the design. */
int pngf_set_design(pngf_handle *h, const uint8_t *bits);

/* Current objective f, outputs x cplx[nfreq] and (optional, may be NULL)
 * design fields e_d cplx[nfreq*n_d].  With PEC pixels e_d holds z: the total
 * field on open pixels, the equivalent current j (design-region field
 * b - G j) on conducting ones. */
int pngf_evaluate(pngf_handle *h, double *f, double *x, double *e_d);

/* Exact objective after flipping each candidate alone from the current state
 * (eq. lru_eobj_rs with M = 1; O(N_d) per candidate).  cand[n] pixel ids,
 * f_new[n] out.  PNGF_EINVAL for ids out of range. */
int pngf_score_flips(pngf_handle *h, const int32_t *cand, int32_t n,
                     double *f_new);

/* Gradient of the objective with respect to the relative permittivity of
 * every pixel at the current design (Supplementary Note 5,
 * eq. supp_grad_chainrule): grad[m] = df/d eps_m = sum_f 2 Re[conj(x_f)
 * dx_f/d eps_m] / (nfreq norm_f) with dx_f/d eps_m = k0^2 E_f[m] R'_f[m]
 * (R' is the adjoint row of the current design).  O(N_d nfreq) from the
 * maintained state, no solve.  grad[n_d] host out.  PNGF_EINVAL for PEC
 * pixels (a conductor has no permittivity to vary). */
int pngf_gradient(pngf_handle *h, double *grad);

/* Accept the flips pix[n] one after another (Sherman-Morrison update of C^-1,
 * E, R' and x; eq. lru_woodbury with M = 1). */
int pngf_accept_flips(pngf_handle *h, const int32_t *pix, int32_t n);

/* Flip the distinct pixels pix[n] together: one exact block-Woodbury update
 * of C^-1 per 64 pixels (eq. lru_woodbury with M = n, on the matrix cores),
 * then E, R' and x re-formed from C^-1 (three matrix passes).  This is the
 * sparse design update of a level-set step (Supplementary Note 6: the M
 * pixels that cross the boundary change at once).  FP64_PLAIN or RFORM
 * handles; PNGF_EINVAL for MIXED, ids out of range or repeated. */
int pngf_flip_set(pngf_handle *h, const int32_t *pix, int32_t n);

/* Re-form C^-1 from G and the current design by FP64 LU (direct re-inversion,
 * Results, Computational efficiency), with one step of iterative refinement of
 * E against C. */
int pngf_refresh(pngf_handle *h);

/* Direct binary search on the device (Results, Direct binary search):
 * perms[n_sweeps*n_d] are the visiting orders of the sweeps; a flip is kept
 * iff f' - f > eta f; after a keep the sweep continues at the next position;
 * the run stops when a whole sweep keeps nothing (converged), after n_sweeps
 * sweeps, or after max_accepts keeps.  accepted[max_accepts] receives the
 * kept pixels, f_trace[max_accepts] the objective after each (either may be
 * NULL).  Starts from the design set by pngf_set_design. */
int pngf_dbs_run(pngf_handle *h, const int32_t *perms, int32_t n_sweeps,
                 int32_t *accepted, double *f_trace, pngf_dbs_result *res);

/* Direct binary search over tiles: groups of pixels flipped together, the
 * paper's multi-DOF tiles (M field components per tile) and symmetry-tied
 * tile groups, a rank-M update (eq. lru_dcn).  tiles[n_tiles*m] holds each
 * tile's pixel ids, distinct within a tile, padded at the end with -1 (at
 * least one id per tile); perms[n_sweeps*n_tiles] order the tiles per sweep.
 * Every tile is scored exactly from the current FP64 state by the rank-M
 * Woodbury identity (eqs. lru_woodbury, lru_eobj_rs: an M x M block of
 * C^-1 G and an M x M solve per tile); the first improving tile in visiting
 * order (f' - f > eta f) is accepted by a block-Woodbury update of C^-1 on
 * the matrix cores, after which E, R' and x are re-formed.  Sweep,
 * convergence and stop rules as pngf_dbs_run; accepted[] receives tile ids.
 * Needs an FP64_PLAIN handle bound with max_tile >= m, 1 <= m <= 64,
 * 1 <= n_tiles <= n_d, n_tiles * Mpad^2 <= 512 n_d (Mpad = 16, 32 or 64, the
 * smallest >= m), n_sweeps <= max_sweeps; PNGF_EINVAL otherwise. */
int pngf_tile_dbs_run(pngf_handle *h, const int32_t *tiles, int32_t n_tiles, int32_t m,
                      const int32_t *perms, int32_t n_sweeps, int32_t *accepted,
                      double *f_trace, pngf_dbs_result *res);

/* Total device time (ms, HIP events on the bound stream; needs
 * PNGF_FLAG_TIMING, or PNGF_FLAG_TIMING_STEPS for id 2 only) and launch
 * count of the kernels of the last pngf_dbs_run (for id 2 of a persistent
 * mixed search: its accepted steps),
 * per kernel id: 0 full scoring pass, 1 select, 2 accept (+ rescore),
 * 3 FP64 inversion, 4 other re-inversion work (GEMVs, outputs), 5 panel fold,
 * 6 mixed-path q row, 7 FP64 block-Woodbury update (mixed refresh, tile
 * accept), 8 tile scoring. */
int pngf_kernel_times(pngf_handle *h, int32_t kernel_id, double *total_ms,
                      int64_t *launches);

/* Bound of the persistent mixed search's grid-barrier waits: a workgroup
 * polls at most `polls` times (default 1 << 20, about a second) before it
 * gives up; the search then fails with PNGF_ENUMERIC, the barrier words are
 * cleared, and the handle needs pngf_set_design before its next search.  For
 * devices shared with other work and for tests of that path.  PNGF_EINVAL
 * unless polls >= 1. */
int pngf_set_persist_spin(pngf_handle *h, int32_t polls);

/* Bound of the probe residual that an inversion without row exchanges must
 * meet (see PNGF_FLAG_PIVOT_SEARCH; default 1e-12).  tol = 0 sends every
 * inversion to the pivot search, for tests of that path.  PNGF_EINVAL
 * unless tol >= 0. */
int pngf_set_inverse_check(pngf_handle *h, double tol);

/* Counts of the FP64 inversions this handle finished without row exchanges
 * and with the pivot search (either pointer may be NULL). */
int pngf_inverse_stats(pngf_handle *h, int64_t *unpivoted, int64_t *pivoted);

/* For tests of the recovery path: the next n FP64 block-Woodbury refreshes
 * of the mixed search report their capacitance matrix as singular, so the
 * search re-inverts C^-1 instead (as it does for a truly singular one; with
 * the persistent search that check happens at the next launch, which then
 * runs no step).  The search's results do not change.  PNGF_EINVAL unless
 * n >= 0. */
int pngf_force_singular_refresh(pngf_handle *h, int32_t n);

int pngf_destroy(pngf_handle *h);

/* ---- batches (many independent problems advanced together) -------------
 * The per-frequency and per-design systems are independent (Results,
 * Computational efficiency), so a batch advances every problem by one DBS
 * step per launch: one workgroup per row of every active problem (or a
 * persistent grid striding over them), captured as a hipGraph of 6 steps
 * that is replayed until every problem has converged.  FP64 refreshes
 * (MIXED) are done per problem between replays: a problem that asks for one
 * skips a round while its refresh runs on one of four internal streams
 * (created by pngf_batch_bind, default priority), beside the other problems'
 * steps; all of their work is joined to the batch stream before
 * pngf_batch_dbs_run returns.  Results equal the solo pngf_dbs_run of each
 * problem (same accepted sequences; MIXED objective traces to FP32 rounding,
 * final objectives to FP64 rounding). */
typedef struct pngf_batch pngf_batch;

/* handles[n]: distinct, each bound (same precision, same stream) before
 * pngf_batch_bind; each needs pngf_set_design before pngf_batch_dbs_run.
 * The batch does not own the handles. */
int pngf_batch_create(pngf_handle *const *handles, int32_t n, pngf_batch **out);
const char *pngf_batch_last_error(const pngf_batch *b);

/* Device bytes of the batch workspace (problem descriptors and states). */
int pngf_batch_workspace_bytes(pngf_batch *b, size_t *bytes);

/* Bind caller-owned device memory (256-byte aligned) and the stream every
 * handle is bound to; it must not be the legacy default stream (the steps are
 * captured as a hipGraph).  PNGF_EINVAL otherwise.  The first bind creates
 * the batch's refresh streams (released by pngf_batch_destroy). */
int pngf_batch_bind(pngf_batch *b, void *dev_ws, size_t bytes, void *hip_stream);

/* Launch shape: 0 = one workgroup per row, g > 0 = persistent grid of g
 * workgroups (the autotuner's choice can be stored and set here). */
int pngf_batch_set_grid(pngf_batch *b, int32_t grid);

/* Run DBS on every problem: perms[p] / n_sweeps[p] as for pngf_dbs_run;
 * accepted[p], f_trace[p] (capacity max_accepts of handle p, may be NULL) and
 * results[p] receive each problem's outcome.  autotune != 0 times the
 * candidate launch shapes (grid sizes; for MIXED handles also work items of
 * eight or four rows) on the first replays (identical arithmetic), one shape
 * per round, and keeps the fastest per streamed matrix entry (a round's time
 * over the sum of N_d^2 x frequencies of its active problems, since problems
 * sit out rounds for their refreshes); pngf_batch_tuning reports the
 * timings. */
int pngf_batch_dbs_run(pngf_batch *b, const int32_t *const *perms, const int32_t *n_sweeps,
                       int32_t *const *accepted, double *const *f_trace,
                       pngf_dbs_result *results, int32_t autotune);

/* Autotuner record of the last run, one entry per launch shape tried:
 * grids[k] (0 = one workgroup per work item), rows[k] (rows per work item:
 * 8 or 4 for MIXED handles, 1 for FP64 rows) and device ms per step; any of
 * the arrays may be NULL, *n receives the number of entries. */
int pngf_batch_tuning(pngf_batch *b, int32_t *grids, int32_t *rows, double *ms_per_step,
                      int32_t cap, int32_t *n);

/* Device ms per batched step of the last replay (HIP events). */
int pngf_batch_ms_per_step(pngf_batch *b, double *ms);

int pngf_batch_destroy(pngf_batch *b);

/* ---- learned flip proposal ------------------------------------------------
 * Not in the paper, which contrasts PNGF's exact evaluations with surrogate
 * models: here a network only ORDERS the exact PNGF evaluations
 * (eq. lru_eobj_rs) and never decides a flip.
 *
 * Inputs, seven channels per pixel of an H x W design region (pixel m at row
 * m / W, column m % W), from the current state at the first frequency:
 *   0 design bit;  1, 2 Re, Im E[m] / max|E|;  3, 4 Re, Im R'[m] / max|R'|;
 *   5 |G_mm| / max|G_mm|;  6 asinh(df_lin[m] / (1e-3 f)), where df_lin is
 *   the flip's objective change with the denominator of eq. lru_eobj_rs set
 *   to 1 (summed over frequencies).  With PEC pixels, E is the z vector of
 *   pngf_evaluate and G the G - I the kernels run on.
 * Network: four 3x3 convolutions, 7 -> 32 -> 32 -> 32 -> 1 channels, zero
 * padding, ReLU between layers; BF16 operands on the matrix cores with FP32
 * accumulation, FP32 master weights, mean Huber loss (delta 1), Adam
 * (0.9, 0.999, 1e-8). */
typedef struct pngf_model pngf_model;

/* He-normal initial weights from seed, zero biases; max_batch images per
 * call.  PNGF_EINVAL unless 1 <= H*W <= 8192 and max_batch >= 1. */
int pngf_model_create(int32_t H, int32_t W, int32_t max_batch, uint64_t seed,
                      pngf_model **out);
/* Message of the last failure of m (of pngf_model_create if m is NULL). */
const char *pngf_model_last_error(const pngf_model *m);
int pngf_model_num_params(pngf_model *m, int32_t *n);
/* Device workspace needed by pngf_model_bind. */
int pngf_model_workspace_bytes(pngf_model *m, size_t *bytes);
/* Bind a caller-owned, 256-byte aligned device workspace and a HIP stream;
 * uploads the current parameters.  The workspace must outlive m. */
int pngf_model_bind(pngf_model *m, void *dev_ws, size_t bytes, void *hip_stream);

/* Flat FP32 parameters [W1, b1, ..., W4, b4], W as [out][in][3][3]; n must
 * equal pngf_model_num_params. */
int pngf_model_get_params(pngf_model *m, float *params, int32_t n);
int pngf_model_set_params(pngf_model *m, const float *params, int32_t n);

/* Host arrays: X[N][7][H][W] in, Y[N][1][H][W] out; 1 <= N <= max_batch. */
int pngf_model_forward(pngf_model *m, const float *X, int32_t N, float *Y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass as pngf_model_forward, with no model object and no workspace.
 * All pointers are device pointers owned by the caller: params[n_params]
 * (the flat FP32 parameters, as pngf_model_get_params lays them out),
 * X[N][7][H][W] in, Y[N][1][H][W] out.  Work is queued on hip_stream (no
 * wait).  Its packed weights and activations live in a file-scope device
 * array of 4 MiB + 64 KiB per GPU, kept until the process ends: N*H*W must
 * not exceed 16384 pixels (PNGF_EINVAL otherwise).  Calls on one GPU share
 * that array, so calls that overlap in time on one GPU (different streams,
 * threads or processes' streams on it) race; each call clears and rewrites
 * what it reads.  Calls no hipMalloc, hipFree or allocating library routine.
 * Errors: PNGF_EINVAL for null pointers, sizes out of range or a parameter
 * count that does not match the network; PNGF_EDEVICE for HIP errors
 * (message: pngf_model_last_error(NULL)). */
int pngf_model_forward_noalloc(const float *params, int32_t n_params, const float *X,
                               int32_t N, int32_t H, int32_t W, float *Y, void *hip_stream);

/* One step on a batch: forward, mean Huber loss against T[N][1][H][W],
 * backward; grads (optional, num_params floats) receive the gradient; an
 * Adam update with learning rate lr if lr > 0.  *loss = mean loss before the
 * update. */
int pngf_model_train_step(pngf_model *m, const float *X, const float *T, int32_t N, float lr,
                          double *loss, float *grads);
int pngf_model_destroy(pngf_model *m);

/* The seven input channels of the current state of h (X[7][n_d], host
 * float), for logging training pairs.  PNGF_EINVAL unless the design region
 * is a full rectangle. */
int pngf_features(pngf_handle *h, float *X);

/* Ranked search.  Per state every pixel is ranked, by the network m (which
 * must be bound to h's stream and sized to the design) or, with m NULL, by
 * channel 6 above (the first-order change); the ranking is scored exactly k
 * pixels at a time, best first, and the best improving pixel (f' - f > eta
 * f) of the first chunk that has one is accepted (a Sherman-Morrison update,
 * eq. lru_woodbury with M = 1).  Converged when the whole ranking holds no
 * improving pixel; stops after max_accepts accepts.
 *   k = 1 (the first improving pixel of the ranking) runs on the device for
 *   every precision: the search steps of pngf_dbs_run with the visiting
 *   order replaced by the state's ranking (re-ranked after every accept, all
 *   frequencies in each launch, no host round trip per state); the mixed
 *   form decides in FP64 inside its error band, so every accept is exact.
 *   max_accepts <= the bound options' max_accepts.
 *   k > 1 needs an FP64 plain handle (chunks scored from the host).
 * accepted / f_trace (optional, max_accepts entries) receive the pixels and
 * objectives; res->attempts counts the exact evaluations performed (ranked
 * positions up to the accepted one, all n_d at convergence), res->sweeps the
 * chunks scored beyond the first of each state.  Needs a rectangular design,
 * n_d <= 8192 and 1 <= k <= n_d. */
int pngf_learned_dbs_run(pngf_handle *h, pngf_model *m, int32_t k, int32_t max_accepts,
                         int32_t *accepted, double *f_trace, pngf_dbs_result *res);

#ifdef __cplusplus
}
#endif

#endif /* PNGF_H */
