/*
 * spgm.h -- C ABI of libspgm.so, the MI355X (gfx950) matrix-free stochastic projector for
 * l1-regularised near-field MIMO imaging with the stochastic proximal gradient method
 * (O. Oral, arXiv 2509.00774).
 *
 * Model (Sec. II, Eqs. 1-2): measurements y in C^M, reflectivity s in C^N, y = A s + w with
 *     A_{m,n} = p(f_m) exp(-j 2 pi f_m (|r_Tm - r_n| + |r_Rm - r_n|) / c) / (4 pi |r_Tm - r_n| |r_Rm - r_n|).
 * The library never stores A: every call forms the entries it needs on the GPU.
 *
 * Conventions shared by every entry point
 *   - complex numbers are complex64: interleaved (re, im) float32, the layout of torch.complex64;
 *   - measurement index m = (i_f * T + i_t) * R + i_r, 0 <= m < M = F*T*R;
 *   - voxel index n = (i_z * ny + i_y) * nx + i_x, 0 <= n < N = nx*ny*nz, voxel centre
 *     r_n = centre + (i - (n_axis - 1)/2) * pitch on each axis;
 *   - a minibatch is `rows`: B measurement indices (int32, device memory).  Rows may repeat;
 *     a repeated row counts once per occurrence, as in the sum of Eq. 6;
 *   - pointers named *_d are device pointers owned by the caller and must stay valid until
 *     the work queued on `stream` has finished; `stream` is a hipStream_t (NULL = the null
 *     stream).  Calls are asynchronous with respect to the host unless stated otherwise;
 *   - every call returns an spgm_status code and never throws; spgm_last_error() gives a
 *     message for the most recent failure on the calling thread;
 *   - a plan belongs to the device that was current when it was created; calls switch to that
 *     device for their duration;
 *   - calls on one plan are not thread-safe and must not overlap on different streams (the
 *     plan's workspace is shared); distinct plans are independent.
 */
#ifndef SPGM_H
#define SPGM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spgm_status {
    SPGM_OK = 0,
    SPGM_E_INVALID = 1,      /* bad argument: null pointer, size out of range, bad geometry */
    SPGM_E_NOMEM = 2,        /* device allocation failed */
    SPGM_E_DEVICE = 3,       /* HIP runtime error (no device, launch failure, ...) */
    SPGM_E_NONFINITE = 4,    /* a non-finite iterate was detected (spgm_solve_tol) */
    SPGM_E_UNSUPPORTED = 5,  /* valid request outside what the kernels support */
    SPGM_E_BADROW = 6        /* a row index outside [0, M) was seen on the device (sticky) */
} spgm_status;

/* How the phase f_m (d_T + d_R)/c, hundreds of turns, is brought to float32 before sin/cos. */
typedef enum spgm_phase_mode {
    /* Default.  Per voxel tile, the reference round trip of every row is formed and reduced
     * modulo one turn in float64; each voxel adds its small offset from the tile centre,
     * computed in float32 from the exact difference of squared distances. */
    SPGM_PHASE_COMP32 = 0,
    /* Distances and phase in float64, reduced modulo one turn in float64, then float32 sin/cos. */
    SPGM_PHASE_F64 = 1,
    /* Uncompensated float32 distances and phase (reference for the precision study). */
    SPGM_PHASE_NAIVE32 = 2
} spgm_phase_mode;

/* Imaging geometry (Sec. II).  Host pointers; the plan copies what it needs, so the caller may
 * free them after spgm_plan_create returns. */
typedef struct spgm_geometry {
    int32_t n_tx, n_rx, n_freq;   /* T, R, F (each >= 1) */
    int32_t nx, ny, nz;           /* voxel grid (each >= 1) */
    const double *tx_xyz;         /* T x 3 transmitter positions r_T (m) */
    const double *rx_xyz;         /* R x 3 receiver positions r_R (m) */
    const double *freq_hz;        /* F frequencies f (Hz), > 0 */
    const double *pulse;          /* F x 2 (re, im) pulse spectrum p(f); NULL means p = 1 */
    double centre[3];             /* grid centre (m) */
    double pitch[3];              /* voxel pitch (m), each > 0 */
    double c;                     /* propagation speed (m/s), > 0 */
} spgm_geometry;

typedef struct spgm_plan spgm_plan;

/* Largest |argument| of sin/cos, in turns, that the compensated float32 phase (SPGM_PHASE_COMP32)
 * can form for `geom` (Sec. II, Eq. 2, the phase f (d_T + d_R)/c): the per-tile reference phase
 * is reduced to [-1/2, 1/2] in float64 and each voxel adds f/c (delta_T + delta_R), where each
 * delta is the antenna's distance to the voxel minus its distance to the centre of the 8 x 8 x 4
 * voxel brick, at most the brick's half-diagonal h; so *turns = 1/2 + 2 max_f (f/c) h.  The
 * float32 argument carries a rounding error of half a unit in its last place, which grows with
 * this bound; the kernels' accuracy was characterised for arguments within
 * SPGM_COMP32_WINDOW_TURNS, and spgm_plan_create refuses COMP32 plans beyond it.  Host only: needs
 * no device.  SPGM_E_INVALID for a NULL pointer, a count < 1, or a pitch, c or frequency that is
 * not finite and > 0. */
#define SPGM_COMP32_WINDOW_TURNS 8.0
int spgm_phase_window(const spgm_geometry *geom, double *turns);

/* Create a plan for `geom` on the current HIP device (Sec. II, Eq. 2 defines what it encodes).
 * Rejects (SPGM_E_INVALID): null pointers, any count < 1, M or N above 2^31 - 1, pitch or c or a
 * frequency <= 0, a non-finite value, or a voxel closer than 1e-9 m to an antenna (Eq. 2 is
 * singular there).  SPGM_E_UNSUPPORTED: min(T, R) > 64 or T + R > 512, or phase_mode
 * SPGM_PHASE_COMP32 with spgm_phase_window above SPGM_COMP32_WINDOW_TURNS (a pitch too coarse for
 * the highest frequency; SPGM_PHASE_F64 has no such limit).  On success *out owns device memory
 * released by spgm_plan_destroy.  Synchronous. */
int spgm_plan_create(spgm_plan **out, const spgm_geometry *geom, int32_t phase_mode);

/* Options of spgm_plan_create_ex (spgm_plan_opts_init: phase_mode SPGM_PHASE_COMP32, device -1,
 * tune_cache NULL). */
typedef struct spgm_plan_opts {
    int32_t phase_mode;     /* a spgm_phase_mode */
    int32_t device;         /* HIP device ordinal the plan lives on; -1: the current device */
    const char *tune_cache; /* default cache file of this plan's autotuners (copied; NULL: none, so
                               the autotuners use SPGM_TUNE_CACHE) */
} spgm_plan_opts;

int spgm_plan_opts_init(spgm_plan_opts *opts);

/* spgm_plan_create with options: creates the plan on opts->device (which must exist:
 * SPGM_E_INVALID otherwise; the calling thread's current device is left as it was) and records
 * the autotuner cache file.  Same geometry checks and errors as spgm_plan_create. */
int spgm_plan_create_ex(spgm_plan **out, const spgm_geometry *geometry, const spgm_plan_opts *opts);

/* Release a plan and its device memory (NULL is a no-op).  Synchronises the plan's device. */
int spgm_plan_destroy(spgm_plan *plan);

/* M = F*T*R and N = nx*ny*nz of the plan (either output pointer may be NULL). */
int spgm_plan_dims(const spgm_plan *plan, int64_t *M, int64_t *N);

/* Forward projection of the minibatch (Sec. II, Eq. 1 restricted to rows, Sec. IV-A):
 *     y_d[j] = sum_n A_{rows_d[j], n} s_d[n],  j < B.
 * rows_d: int32[B]; s_d: complex64[N]; y_d: complex64[B] (output, may not alias s_d).
 * 1 <= B <= 2^24.  May grow the plan's workspace (hipMalloc, synchronous) on first use of a
 * larger B. */
int spgm_forward(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *s_d, void *y_d,
                 void *stream);

/* Adjoint (conjugate-transpose) projection of the minibatch, unscaled:
 *     g_d[n] = sum_j conj(A_{rows_d[j], n}) r_d[j],  n < N.
 * r_d: complex64[B]; g_d: complex64[N] (output).  Same limits as spgm_forward. */
int spgm_adjoint(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *r_d, void *g_d,
                 void *stream);

/* One SPGM iteration (Sec. IV, Eq. 5 with the minibatch gradient of Eq. 6), in place:
 *     s <- S_alpha( s - (eta/B) A_B^H (A_B s - y_B) ),  S_a(v) = v max(0, 1 - a/|v|),
 * where y_B gathers y_d at rows_d and alpha = lambda * eta.  y_d: complex64[M] (full
 * measurement vector); s_d: complex64[N] in/out.  eta > 0, alpha >= 0, finite. */
int spgm_step(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *y_d, void *s_d,
              float eta, float alpha, void *stream);

/* spgm_step that also writes g_d = A_B^H (A_B s - y_B) at the entering iterate (unscaled, the
 * minibatch gradient of Eq. 6 times B; complex64[N], must not alias s_d): the quantity the
 * backward of an unrolled iteration needs, formed by the same column reduction.  The update
 * of s_d is bitwise that of spgm_step. */
int spgm_step_grad(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *y_d, void *s_d,
                   float eta, float alpha, void *g_d, void *stream);

/* spgm_step for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and launch shapes as
 * spgm_step, so the same result bit for bit, with the step's workspace (sorted rows, forward
 * partials, scaled residuals, adjoint partials) carved from a fixed 64 MiB device array that the
 * library holds on every GPU it runs on until the process ends; the call itself allocates
 * nothing.  The plan (created beforehand) supplies the geometry.  Workspace needed:
 * 16 B + 8 B x (voxel bricks + 1) per row plus 8 B x N x (adjoint row splits), each rounded up to
 * 256 B; above 64 MiB the call fails with SPGM_E_UNSUPPORTED (about B = 15 000 rows on a
 * 64 x 64 x 32 grid, 1 800 on a 128 x 128 x 64 grid; spgm_step has no such limit).  Every call on one GPU uses that GPU's one
 * array: calls that overlap on one GPU (other streams, other threads, other plans) race and must
 * be serialised by the caller.  Arguments and errors as spgm_step. */
int spgm_step_noalloc(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *y_d, void *s_d,
                      float eta, float alpha, void *stream);

/* `iters` SPGM iterations; iteration k uses rows_d[k*B .. k*B + B - 1] (rows_d: int32[iters*B]).
 * Bitwise equal to `iters` calls of spgm_step.  iters >= 0.  Intermediate iterates alternate
 * between s_d and a plan-owned buffer of N complex64 (allocated on the first solve); s_d holds
 * the result when the call's work on `stream` is complete. */
int spgm_solve(spgm_plan *plan, const int32_t *rows_d, int32_t iters, int32_t B, const void *y_d,
               void *s_d, float eta, float alpha, void *stream);

/* spgm_solve executed as a HIP graph: the sort and the launches of all `iters` iterations are
 * captured once (on a stream owned by the plan) and the instantiated graph is replayed on
 * `stream`.  The graph is kept for the next call and replayed as long as rows_d, iters, B, y_d,
 * s_d, eta and alpha are the same (the buffers' contents may change between calls, as in
 * repeated solves on new measurements); any other arguments re-capture it.  The first call
 * pays the capture and instantiation cost.  Same results as spgm_solve, bit for bit. */
int spgm_solve_graph(spgm_plan *plan, const int32_t *rows_d, int32_t iters, int32_t B, const void *y_d,
                     void *s_d, float eta, float alpha, void *stream);

/* spgm_solve until the termination rule of the experiments (Sec. V: the change in reflectivity
 * magnitudes falls below a threshold), read as the relative 2-norm change
 *     || |s^k| - |s^{k-1}| ||_2  <  tol || |s^{k-1}| ||_2,
 * evaluated after every iteration k = 1, 2, ... (never met while s^{k-1} = 0).  The two sums are
 * formed on the device in float64 in a fixed order.  Iterations are queued in groups of
 * check_every (>= 1); after each group the host reads the group's records (one synchronisation
 * per group) and, if the rule was met inside it, the iterate is brought back to the group's
 * first iterate and advanced to the stopping iteration with the same kernels on the same rows,
 * so s_d ends bitwise at the iterate the rule was met at (the same as spgm_solve with that many
 * iterations).  tol <= 0 runs all `iters` iterations.  use_graph = 1 replays each full group as
 * one captured HIP graph (kept while check_every, B, y_d, s_d, eta and alpha are unchanged).
 * On return *iters_done is the number of iterations performed (the stopping k, or iters) and, if
 * `changes` (host double[iters]) is not NULL, changes[k-1] holds the relative change of each
 * performed iteration (+inf while s^{k-1} = 0).  Synchronous: returns after the stop is known.
 * SPGM_E_NONFINITE: an iteration produced a non-finite change (a non-finite iterate); it stops
 * there and *iters_done names it.  Other errors as spgm_solve. */
int spgm_solve_tol(spgm_plan *plan, const int32_t *rows_d, int32_t iters, int32_t B, const void *y_d,
                   void *s_d, float eta, float alpha, double tol, int32_t check_every, int32_t use_graph,
                   int32_t *iters_done, double *changes, void *stream);

/* Seeded minibatches (Sec. IV: each SPGM iteration draws its minibatch of rows uniformly at
 * random).  The generator is SplitMix64 (Steele, Lea and Flood, OOPSLA 2014: state += 0x9E3779B9
 * 7F4A7C15; z = state; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9; z = (z ^ z>>27) *
 * 0x94D049BB133111EB; output z ^ z>>31).  Iteration k (global index: start_iter + i) takes
 * outputs u_1, u_2, ... number k 2^32 + 1, k 2^32 + 2, ... of the sequence whose initial state is
 * `seed`, i.e. it starts from state seed + k 2^32 0x9E3779B97F4A7C15 (mod 2^64).  A partial
 * Fisher-Yates shuffle of the identity 0 .. n-1 turns draws into m distinct indices: for
 * j = 0 .. m-1, position j is swapped with position j + floor((u_{j+1} >> 32) (n - j) / 2^32) and
 * index j is the value position j then holds.  Uniform rows: n = M, m = B.  Structured subsets
 * (Sec. IV-A): the same iteration stream draws nf of F frequencies, then nt of T transmitters,
 * then nr of R receivers.  Host only, no device memory. */
int spgm_rows_generate(uint64_t seed, int32_t start_iter, int32_t iters, int64_t M, int32_t B,
                       int32_t *rows_out /* host int32[iters][B] */);
int spgm_subsets_generate(uint64_t seed, int32_t start_iter, int32_t iters, int32_t F, int32_t T, int32_t R,
                          int32_t nf, int32_t nt, int32_t nr, int32_t *f_out /* host int32[iters][nf] */,
                          int32_t *t_out /* host int32[iters][nt] */, int32_t *r_out /* host int32[iters][nr] */);

/* Options of spgm_solve_ex (initialise with spgm_solve_opts_init, then set fields). */
typedef struct spgm_solve_opts {
    int32_t iters;         /* iterations to run, >= 0 */
    int32_t B;             /* rows per minibatch (sampling 0), 1 <= B <= 2^24 (and <= M when drawn) */
    double lambda;         /* l1 weight of Eq. 3, >= 0 */
    double eta;            /* step size, > 0; the threshold is alpha = lambda * eta (Eq. 5) */
    const int32_t *rows_d; /* device int32[iters][B] minibatches, or NULL: drawn by the generator */
    uint64_t seed;         /* generator seed (rows_d == NULL) */
    int32_t sampling;      /* 0: uniform rows; 1: structured subsets (nf x nt x nr, generator only) */
    int32_t nf, nt, nr;    /* structured subset sizes (sampling 1) */
    int32_t start_iter;    /* global index of the first iteration (generator stream), >= 0 */
    double tol;            /* > 0: stop at the termination rule as spgm_solve_tol; 0: all iterations */
    int32_t check_every;   /* iterations per termination check (tol > 0); default 50 */
    int32_t use_graph;     /* 1: replay captured HIP graphs (as spgm_solve_graph / spgm_solve_tol) */
    int32_t *iters_done;   /* optional host out: iterations performed */
} spgm_solve_opts;

/* Defaults: every field zero except check_every = 50. */
int spgm_solve_opts_init(spgm_solve_opts *opts);

/* SPGM solve (Eq. 5 iterated) with options: the minibatches are opts->rows_d or drawn by the
 * generator above for iterations start_iter .. start_iter + iters - 1 (so a solve split over
 * several calls with matching start_iter reproduces one call bit for bit); uniform rows run as
 * spgm_solve, spgm_solve_graph (use_graph) or spgm_solve_tol (tol > 0); structured subsets run as
 * spgm_solve_structured (fixed iterations, no graph: SPGM_E_UNSUPPORTED otherwise).  Drawn
 * minibatches are made on the host in chunks of up to 2^22 rows, copied to a device buffer the
 * plan keeps (through two pinned host buffers, so drawing the next chunk overlaps the device
 * work) and consumed on `stream`; the call returns when the last chunk is queued (after the stop
 * is known when tol > 0).  Errors as the solve it runs; SPGM_E_INVALID for bad options. */
int spgm_solve_ex(spgm_plan *plan, const void *y_d, void *s_d, const spgm_solve_opts *opts, void *stream);

/* Backward of one unrolled SPGM iteration (differentiation of Eq. 5 with the gradient of
 * Eq. 6 with respect to its input iterate, step size and threshold):
 *     z = s - (eta/B) A_B^H (A_B s - y_B),   s' = S_tau(z)    (S as in spgm_step, tau = alpha).
 * For a real loss L, complex gradients carry dL/dRe + j dL/dIm (the convention of PyTorch).
 * Given s (iterate entering the iteration) and sbar_next = dL/ds', writes
 *     sbar = dL/ds = zbar - (eta/B) A_B^H A_B zbar,
 *     zbar = (1 - tau/|z|) sbar' + (tau/|z|) u Re(conj(u) sbar')  where |z| > tau (u = z/|z|), else 0,
 *     *eta_bar = dL/deta = -(1/B) Re <zbar, A_B^H (A_B s - y_B)>,
 *     *tau_bar = dL/dtau = -sum_{|z| > tau} Re(conj(u) sbar').
 * y_d: complex64[M]; s_d, sbar_next_d, sbar_d: complex64[N] (sbar_d may alias sbar_next_d);
 * eta_bar_d, tau_bar_d: device double[1] each (overwritten).  eta > 0, tau >= 0.  The entries
 * of A_B are recomputed (the iterate s is the only state kept from the forward pass). */
int spgm_unrolled_vjp_step(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *y_d,
                           const void *s_d, float eta, float tau, const void *sbar_next_d,
                           void *sbar_d, double *eta_bar_d, double *tau_bar_d, void *stream);

/* spgm_unrolled_vjp_step given the gradient at the entering iterate instead of y:
 * g_d = A_B^H (A_B s - y_B) (unscaled, complex64[N], e.g. from spgm_step_grad when the iterate
 * was recomputed), so only A_B^H A_B zbar forms entries (two passes instead of four).  Same
 * outputs, bit for bit, as spgm_unrolled_vjp_step with the y that gives this g. */
int spgm_unrolled_vjp_step_g(spgm_plan *plan, const int32_t *rows_d, int32_t B, const void *s_d,
                             const void *g_d, float eta, float tau, const void *sbar_next_d,
                             void *sbar_d, double *eta_bar_d, double *tau_bar_d, void *stream);

/* Autotuner.  For minibatch size B, times the forward-tile and adjoint-tile kernels over the
 * candidate launch shapes -- row splits (rows of the minibatch per work-group: splits 1, 2, 3, 4,
 * 6, 8, ... up to ceil(B/64)) times 8 or 16 waves per work-group (16 only where its LDS fits) --
 * on uniform pseudo-random rows, and keeps the fastest shape per kernel for every later call of
 * this plan with this B.  Without tuning, a plan uses 8 waves where two work-groups fit in one
 * compute unit's LDS and 16 otherwise (four waves per SIMD either way).  Results are cached in a JSON file (cache_path, else the
 * environment variable SPGM_TUNE_CACHE, else no file) keyed by GPU architecture, phase mode,
 * T, R, F, grid and B; a cached key is applied without timing.  Writes the chosen splits to
 * *fwd_splits / *adj_splits (either may be NULL).  Synchronous: first waits for all work on the
 * plan's device (the timing rewrites the plan's workspace); allocates temporary device memory.
 * The adjoint's summation order depends on its split, so results may differ from an
 * untuned plan in the last bits (within the parity tolerance). */
int spgm_plan_autotune(spgm_plan *plan, int32_t B, const char *cache_path, int32_t *fwd_splits,
                       int32_t *adj_splits);

/* Autotuner of the shared-geometry batch kernels (spgm_forward_batched and the calls built on
 * it) for minibatches of B rows and the given spgm_mm_precision.  The forward candidates are
 * every combination that fits of: row tiles per wave nrt = 1..4; 8 waves over whole bricks or
 * (A-operand-order form only) 4 waves over two z slices per work-group; bricks per work-group
 * half, equal to and twice the default.  The adjoint candidates are row splits of 1, 2 and 4
 * times the default, each staging all of a work-group's rows at once, 256 or 64 rows per group
 * and round.  Each side is timed on pseudo-random rows and right-hand sides and the fastest kept
 * for every later batched call of this plan with this B.  Cached in the same JSON file as
 * spgm_plan_autotune (cache_path, else SPGM_TUNE_CACHE, else none), key as there plus "|mm" and
 * the precision, value [nrt, bricks per work-group, waves, z slices, adjoint splits, staged rows,
 * forward ms, adjoint ms]; a cached key is applied without timing, and a cached shape that does
 * not fit the plan falls back to the default.  shape (int32_t[7], required) receives the applied
 * shape as spgm_plan_batched_shape writes it.  Synchronous;
 * waits for all work on the plan's device first; allocates temporary device memory.  Results of
 * every candidate agree with the default shape's to the batched path's error bounds (the
 * adjoint's summation order follows its split). */
int spgm_plan_autotune_batched(spgm_plan *plan, int32_t B, int32_t precision, const char *cache_path,
                               int32_t *shape);

/* Launch shape of the shared-geometry batch kernels for minibatches of B rows (the autotuned one,
 * else the default): shape[0..6] = {row tiles per wave, bricks per work-group, waves per
 * work-group, z slices per work-group, adjoint row splits, adjoint staged rows per group and
 * round, 1 if the forward forms entries in A-operand order else 0}.  Host only. */
int spgm_plan_batched_shape(const spgm_plan *plan, int32_t B, int32_t *shape);

/* The candidates spgm_plan_autotune_batched times for B: forward shapes as int32_t[4] {nrt,
 * bricks per work-group, waves, z slices} into fwd (up to fwd_cap of them), adjoint shapes as
 * int32_t[2] {row splits, staged rows} into adj (up to adj_cap); *n_fwd and *n_adj receive the
 * full counts.  fwd / adj may be NULL to query the counts.  Host only. */
int spgm_plan_batched_candidates(const spgm_plan *plan, int32_t B, int32_t *fwd, int32_t fwd_cap, int32_t *n_fwd,
                                 int32_t *adj, int32_t adj_cap, int32_t *n_adj);

/* Autotuner of the structured-minibatch kernels for subsets of nf frequencies, nt transmitters
 * and nr receivers: times the small-register instances (8 items per thread and 128 voxels, two
 * work-groups per compute unit; only for nt + nr <= 32 and nt <= 16) against the general ones
 * (16 items, one work-group per compute unit) on the forward and adjoint
 * kernels, and keeps the faster for every later structured call of this plan with this
 * (nf, nt, nr).  Cached like spgm_plan_autotune (key plus "|sf|nf..|nt..|nr..", value
 * [items, ms]).  *items (required) receives the applied choice.  Synchronous; waits for all work
 * on the plan's device first; allocates temporary device memory.  Both instances compute the
 * same sums in the same order. */
int spgm_plan_autotune_structured(spgm_plan *plan, int32_t nf, int32_t nt, int32_t nr, const char *cache_path,
                                  int32_t *items);

/* Items per thread and 128 voxels (8 or 16) of the structured kernel instances used for
 * (nf, nt, nr) on this plan.  Host only. */
int spgm_plan_structured_shape(const spgm_plan *plan, int32_t nf, int32_t nt, int32_t nr, int32_t *items);

/* Launch shape the tile kernels use for minibatches of B rows on this plan (the autotuned one,
 * else the default): row splits and waves per work-group of the forward and adjoint tile
 * kernels.  Any output pointer may be NULL.  Host only. */
int spgm_plan_launch_shape(const spgm_plan *plan, int32_t B, int32_t *fwd_splits, int32_t *fwd_waves,
                           int32_t *adj_splits, int32_t *adj_waves);

/* Shared-geometry batches: K right-hand sides (K images of one scene geometry, or K
 * measurement sets) through one set of entries of the minibatch.  Every entry of A_B is
 * formed once per pass of up to 32 right-hand sides (compensated float32 phase as in
 * SPGM_PHASE_COMP32), rounded to the chosen 16-bit type, and contracted with the right-hand
 * sides, also rounded to that type, on the matrix cores with float32 accumulation.  K > 32 is
 * processed in passes of 32.  Every reduction runs in a fixed order (bitwise reproducible).
 * Expected relative error of each output column against exact arithmetic: about 1.6e-3
 * (bfloat16) and 2e-4 (half), from the two roundings of each product.  Only plans created with
 * SPGM_PHASE_COMP32 are supported (SPGM_E_UNSUPPORTED otherwise), and the brick tables must fit
 * in LDS (min(T, R) <= 32 for the forward pass; SPGM_E_UNSUPPORTED otherwise). */
typedef enum spgm_mm_precision {
    /* bfloat16 operands (8 significant bits, float32 range) */
    SPGM_MM_BF16 = 0,
    /* IEEE half operands (11 significant bits); magnitudes of entries times 1, right-hand
     * sides and scaled residuals must stay below 65504 */
    SPGM_MM_FP16 = 1
} spgm_mm_precision;

/* Batched forward projection (Sec. II, Eq. 1 restricted to the minibatch, K images):
 *     Y_d[j][k] = sum_n A_{rows_d[j], n} S_d[n][k],  j < B, k < K.
 * S_d: complex64[N][K] (row-major, the K values of one voxel adjacent); Y_d: complex64[B][K]
 * (output, caller row order).  1 <= B <= 2^24, K >= 1, precision a spgm_mm_precision.  May grow
 * the plan's workspace (hipMalloc, synchronous). */
int spgm_forward_batched(spgm_plan *plan, const int32_t *rows_d, int32_t B, int32_t K, const void *S_d,
                         void *Y_d, int32_t precision, void *stream);

/* Batched adjoint projection, unscaled:  G_d[n][k] = sum_j conj(A_{rows_d[j], n}) R_d[j][k].
 * R_d: complex64[B][K] (caller row order); G_d: complex64[N][K] (output).  Limits as above. */
int spgm_adjoint_batched(spgm_plan *plan, const int32_t *rows_d, int32_t B, int32_t K, const void *R_d,
                         void *G_d, int32_t precision, void *stream);

/* One SPGM iteration (Sec. IV, Eq. 5 with the gradient of Eq. 6) for each of K problems that
 * share the geometry and the minibatch, in place:
 *     S[:, k] <- S_alpha( S[:, k] - (eta/B) A_B^H (A_B S[:, k] - Ymeas[rows, k]) ).
 * Ymeas_d: complex64[M][K] (full measurement vectors, column k for problem k); S_d:
 * complex64[N][K] in/out.  eta > 0, alpha >= 0, finite.  Limits as above. */
int spgm_step_batched(spgm_plan *plan, const int32_t *rows_d, int32_t B, int32_t K, const void *Ymeas_d,
                      void *S_d, float eta, float alpha, int32_t precision, void *stream);

/* `iters` batched SPGM iterations; iteration i uses rows_d[i*B .. i*B + B - 1].  Equivalent to
 * `iters` calls of spgm_step_batched.  iters >= 0. */
int spgm_solve_batched(spgm_plan *plan, const int32_t *rows_d, int32_t iters, int32_t B, int32_t K,
                       const void *Ymeas_d, void *S_d, float eta, float alpha, int32_t precision,
                       void *stream);

/* Structured minibatches (the Cartesian-product minibatches of Sec. IV-A and Sec. V): a
 * frequency subset f_idx (nf entries), a transmitter subset t_idx (nt) and a receiver subset
 * r_idx (nr), device int32 arrays; the minibatch holds the B = nf*nt*nr rows
 *     j = (i*nt + a)*nr + b  ->  m = (f_idx[i]*T + t_idx[a])*R + r_idx[b].
 * Eq. 2 factors over the two antennas of a row, A_{(f,t,r),n} = q_f a_T[f,t,n] a_R[f,r,n] with
 * a_X = exp(-j 2 pi f d_X / c) / d_X and q_f = p(f)/(4 pi), so only nf*(nt+nr)*N factors are formed
 * (compensated float32 phase per antenna) and the per-frequency products run as float32 GEMMs
 * on the matrix cores; results keep float32 accuracy (same tolerance as spgm_forward).
 * 1 <= nt, nr <= 32, 1 <= nf <= 65535, B <= 2^24; indices need not be distinct.  An index outside its
 * range sets the plan's sticky status (SPGM_E_BADROW, read by spgm_plan_status) and is replaced
 * by 0.  Only SPGM_PHASE_COMP32 plans are supported (SPGM_E_UNSUPPORTED otherwise).  May grow
 * the plan's workspace (hipMalloc, synchronous). */

/* y_d[j] = sum_n A_{m_j, n} s_d[n]; s_d: complex64[N]; y_d: complex64[B] (minibatch order). */
int spgm_forward_structured(spgm_plan *plan, const int32_t *f_idx_d, int32_t nf, const int32_t *t_idx_d,
                            int32_t nt, const int32_t *r_idx_d, int32_t nr, const void *s_d, void *y_d,
                            void *stream);

/* g_d[n] = sum_j conj(A_{m_j, n}) r_d[j], unscaled; r_d: complex64[B]; g_d: complex64[N]. */
int spgm_adjoint_structured(spgm_plan *plan, const int32_t *f_idx_d, int32_t nf, const int32_t *t_idx_d,
                            int32_t nt, const int32_t *r_idx_d, int32_t nr, const void *r_d, void *g_d,
                            void *stream);

/* One SPGM iteration (as spgm_step) on the structured minibatch; y_d: complex64[M]. */
int spgm_step_structured(spgm_plan *plan, const int32_t *f_idx_d, int32_t nf, const int32_t *t_idx_d,
                         int32_t nt, const int32_t *r_idx_d, int32_t nr, const void *y_d, void *s_d,
                         float eta, float alpha, void *stream);

/* `iters` iterations; iteration k uses f_idx_d[k*nf ..], t_idx_d[k*nt ..], r_idx_d[k*nr ..]. */
int spgm_solve_structured(spgm_plan *plan, const int32_t *f_idx_d, int32_t nf, const int32_t *t_idx_d,
                          int32_t nt, const int32_t *r_idx_d, int32_t nr, int32_t iters, const void *y_d,
                          void *s_d, float eta, float alpha, void *stream);

/* Other regularisers in place of the l1 norm of Eq. 3 (the extension noted in Sec. III); the
 * prox of Eq. 5 changes, the data-fidelity gradient does not.
 *   SPGM_REG_L1:           R(s) = sum_n |s_n|; prox S_alpha (as spgm_step).
 *   SPGM_REG_ELASTIC_NET:  R(s) = sum_n |s_n| + (mu/2) sum_n |s_n|^2; prox S_alpha(v) / (1 + alpha mu).
 *   SPGM_REG_TV_MAGNITUDE: R(s) = TV(|s|), the isotropic 3-D total variation of the magnitudes with
 *       forward differences on the voxel grid (zero on the upper face of each axis).  The prox keeps
 *       the phase of v and replaces |v| by the minimiser of 1/2 ||u - |v| ||^2 + alpha TV(u) over
 *       u >= 0, approximated by `tv_iters` iterations of fast gradient projection on the dual
 *       (Beck and Teboulle), started from a zero dual at every call (one launch per iteration).
 * mu: finite, >= 0 (elastic net only).  tv_iters: 0 .. 100000 (TV only; 0 or alpha = 0 leave v
 * unchanged).  The TV prox allocates 68 bytes per voxel of plan workspace on first use
 * (hipMalloc, synchronous). */
typedef enum spgm_reg_kind {
    SPGM_REG_L1 = 0,
    SPGM_REG_ELASTIC_NET = 1,
    SPGM_REG_TV_MAGNITUDE = 2
} spgm_reg_kind;

typedef struct spgm_regularizer {
    int32_t kind;      /* spgm_reg_kind */
    float mu;          /* elastic-net weight of the squared norm */
    int32_t tv_iters;  /* dual iterations of the TV prox */
} spgm_regularizer;

/* v_d <- prox_{alpha R}(v_d) in place; v_d: complex64[N]; alpha finite, >= 0. */
int spgm_prox(spgm_plan *plan, const spgm_regularizer *reg, void *v_d, float alpha, void *stream);

/* One SPGM iteration (as spgm_step) with the prox of `reg`:
 *     s <- prox_{alpha R}( s - (eta/B) A_B^H (A_B s - y_B) ). */
int spgm_step_reg(spgm_plan *plan, const spgm_regularizer *reg, const int32_t *rows_d, int32_t B,
                  const void *y_d, void *s_d, float eta, float alpha, void *stream);

/* `iters` calls of spgm_step_reg; iteration k uses rows_d[k*B .. k*B + B - 1]. */
int spgm_solve_reg(spgm_plan *plan, const spgm_regularizer *reg, const int32_t *rows_d, int32_t iters,
                   int32_t B, const void *y_d, void *s_d, float eta, float alpha, void *stream);

/* Ragged batches of independent scenes (each with its own array, band and grid) advanced
 * together: every SPGM iteration of every scene is one launch per phase (sort, forward tile,
 * row reduction, adjoint tile, column reduction with the prox step).  The tile phases walk a
 * work list of (scene, voxel brick, row range) items ordered longest first with persistent
 * work-groups, so scenes of very different sizes share the chip. */
typedef struct spgm_batch spgm_batch;

/* One plan per geometry (geoms: host array of n spgm_geometry, same rules as spgm_plan_create,
 * one phase mode for all).  Synchronous. */
int spgm_batch_create(spgm_batch **out, const spgm_geometry *geoms, int32_t n, int32_t phase_mode);
int spgm_batch_destroy(spgm_batch *batch);

/* The plan of scene i (owned by the batch; usable with every spgm_plan call). */
int spgm_batch_plan(spgm_batch *batch, int32_t i, spgm_plan **plan);

/* `iters` SPGM iterations of every scene (the update of spgm_step).  Host arrays of length n:
 * B[i] rows per minibatch of scene i; rows_d[i] device int32[iters * B[i]] (iteration k uses
 * rows_d[i][k*B[i] ...]); y_d[i] device complex64[M_i]; s_d[i] device complex64[N_i] in/out;
 * eta[i] > 0, alpha[i] >= 0.  use_graph != 0 captures the launches of the whole solve into a
 * HIP graph and launches it once (one submission; same results).  Grows the batch's workspace
 * with hipMalloc when needed.  Waits for earlier work on `stream` before rewriting the batch's
 * descriptors; calls on one batch must not overlap on different streams. */
int spgm_batch_solve(spgm_batch *batch, int32_t iters, const int32_t *B, const int32_t *const *rows_d,
                     const void *const *y_d, void *const *s_d, const float *eta, const float *alpha,
                     int32_t use_graph, void *stream);

/* Launch shape of spgm_batch_solve's tile phases, kept for later solves of this batch.
 * max_workgroups caps the persistent grid that walks the (scene, brick, row range) work list
 * (0: as many work-groups as fit on the chip at once, the default); the result does not depend
 * on it, bit for bit.  rows_per_split is the length of a work item's row range: scene i's
 * minibatch is cut into ceil(B[i] / rows_per_split) ranges whose column partials are summed in
 * range order (0: 1024, the default; otherwise a positive multiple of 64).  Host only. */
int spgm_batch_options(spgm_batch *batch, int32_t max_workgroups, int32_t rows_per_split);

/* Autotuner of the ragged batch: for minibatch sizes B[0..n-1] (one per scene, host array),
 * times one SPGM iteration of the batch with 256, 512, 1024, 2048, 4096, 8192 and 16384 rows
 * per work item (the row split of every scene; spgm_batch_options' rows_per_split) on
 * pseudo-random rows and keeps the fastest for the batch.  Cached like spgm_plan_autotune (key: architecture, phase
 * mode, number of scenes and a hash of every scene's T, R, F, grid and B; value [rows per work
 * item, ms]); a cached key is applied without timing.  *rows_per_split (optional) receives the
 * applied value.  Synchronous; waits for all work on the batch's device first; allocates
 * temporary device memory.  Results follow the split's summation order (within the batch
 * path's error bounds of every other split). */
int spgm_batch_autotune(spgm_batch *batch, const int32_t *B, const char *cache_path, int32_t *rows_per_split);

/* Device-detected row errors of the batch's earlier solves (as spgm_plan_status). */
int spgm_batch_status(spgm_batch *batch, int32_t *status);

/* Device-detected errors of earlier calls (currently SPGM_E_BADROW).  Synchronises the plan's
 * device, writes the sticky status to *status (SPGM_OK if none) and clears it. */
int spgm_plan_status(spgm_plan *plan, int32_t *status);

/* Kernel timing instrumentation.  While enabled, every launch of the two entry-generating
 * kernels (forward tile, adjoint tile) is bracketed by HIP events recorded on the call's
 * stream.  spgm_plan_timing_read synchronises the plan's device, returns the summed kernel
 * durations (milliseconds) and launch counts since the last read, and resets them.  Any
 * output pointer may be NULL.  Launches made through a captured graph (spgm_solve_graph) are
 * not timed. */
int spgm_plan_timing(spgm_plan *plan, int32_t enable);
int spgm_plan_timing_read(spgm_plan *plan, double *fwd_ms, int64_t *fwd_launches, double *adj_ms,
                          int64_t *adj_launches);

/* Issue-rate probe for the rooflines of the entry-generating kernels, on the current device.
 * One launch of 8 work-groups of 256 threads per compute unit, each lane running `iters`
 * rounds of 8 independent dependency chains of: kind 0, v_fma_f32; kind 1, v_sin_f32; kind 2,
 * v_cos_f32; kind 3, the entry body of the tile kernels (one phase FMA, sin, cos and four FMAs
 * of the complex multiply-add).  Writes the chain steps per second over all lanes
 * (*ops_per_s: lane-instructions/s for kinds 0-2, entry bodies/s for kind 3) and the launch
 * time (*ms, may be NULL), timed with HIP events after one warm-up launch.  Synchronous;
 * allocates a small device buffer. */
int spgm_calibrate(int32_t kind, int32_t iters, double *ops_per_s, double *ms);

/* Message describing the last failure of a call on this thread ("" if none). */
const char *spgm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPGM_H */
