/*
 * hmps.h -- C-ABI of libhmps, a multi-level power-series H-matrix solver for
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Negi, Balakrishnan, Rao, "Multi-Level Power Series Solution for
 * Large Surface and Volume Electric Field Integral Equation" (arXiv
 * 2307.03968).  The dense system [Z] x = b (Sec. II, eq. 5) is compressed
 * as an H-matrix Z = Z_N + Z_F (Sec. III, eq. 6): a binary cluster tree, the
 * admissibility test of eq. 7, dense near blocks and ACA-compressed far
 * blocks grouped by level (eq. 8).  The solve splits Z_l = D + R_l, D the
 * leaf self-interaction blocks, R_l the off-diagonal near blocks plus the far
 * blocks of level >= l, and evaluates the truncated power series of
 * Sec. IV (eq. 12-13, 20-22):
 *
 *     x_K = sum_{k=0..K} (-D^{-1} R_l)^k D^{-1} b .
 *
 * Conventions for every call:
 *   - Return value: HM_OK (0) on success, > 0 a state or warning, < 0 an
 *     error; hm_last_error() gives a message for the calling thread.
 *   - Vectors are complex128 (interleaved re, im doubles), column-major
 *     n x nrhs with leading dimension ld >= n, in ORIGINAL point order.
 *   - *_dev pointers are device pointers on the current HIP device; a
 *     hip_stream argument is a hipStream_t (NULL = the null stream).  Device
 *     calls are stream-ordered and asynchronous unless stated otherwise.
 *   - The library copies every host input it is given; the caller keeps
 *     ownership of its buffers.  An hm_matrix_t owns all device memory of
 *     one geometry until hmat_free.  Calls on one handle are not
 *     thread-safe (use one handle per stream); server calls are.
 *   - There is no CPU fallback: a device call without a usable gfx950
 *     device fails with HM_EHIP.
 */
#ifndef HMPS_H
#define HMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HM_OK         0
#define HM_ENOTREADY  1   /* ps_poll: the request has not finished          */
#define HM_EDIVERGED  2   /* a result was written but the series grew       */
                          /* (||y_K|| > ||y_0||) or went non-finite          */
#define HM_EINVAL    (-1) /* bad argument                                    */
#define HM_ENOMEM    (-2) /* device allocation failed or over the budget     */
#define HM_EHIP      (-3) /* HIP runtime error (no device, launch failure)   */
#define HM_EBUSY     (-4) /* no server slot free; retry                      */
#define HM_ESTATE    (-5) /* handle not in a state that allows this call     */

/* ---- enums --------------------------------------------------------------- */
enum { HM_SURFACE = 0, HM_VOLUME = 1 };
/* HM_F64: every product in FP64.  HM_F32_APPLY: near and far products read
 * FP32 copies of the blocks (FP64 vectors and accumulation); leaf LU,
 * D^{-1}, residuals and refinement stay FP64. */
enum { HM_F64 = 0, HM_F32_APPLY = 1 };
/* PS_SERIES: return x_K.  PS_REFINE: x <- x + P_K(b - Z_l x) passes (P_K is
 * the K-term series operator, residual in FP64) until the correction is
 * below refine_tol relative to x (or until its norm has grown five passes in a
 * row: the series does not contract, reported as diverged); the fixed
 * point is Z_l^{-1} b and the per-pass error factor is rho(D^{-1} R_l)^{K+1}.  PS_REFINE_FIXED: exactly
 * max_passes such passes with no host synchronisation (refine_tol only
 * decides the diverged flag of the statistics).  PS_SERIES and
 * PS_REFINE_FIXED without statistics only enqueue device work: once a
 * first call with the same nrhs has sized the workspace, a call can be
 * recorded by stream capture into a HIP graph and replayed.  Such a graph
 * refers to the handle's workspace and work lists: it stays valid until
 * hmat_free, a call with more right-hand sides than any before the capture
 * (the workspace grows), or a change of term_wgs (hmat_tune,
 * hmat_autotune), whichever comes first.
 * Norm-based quantities (growth, ||d|| / ||x||) are taken per instance of a
 * batched handle and the maximum over instances is reported. */
/* PS_GMRES: restarted GMRES on Z_l x = b (FP64 products with Z_l, two
 * classical Gram-Schmidt passes per step) with the K-term series as right
 * preconditioner in the flexible form x = sum_j (P_K v_j) y_j; precision
 * selects the block copies the preconditioner reads.  K = 0 preconditions
 * with D^{-1} alone (block Jacobi), which suits rho(D^{-1} R_l) >= 1, where
 * the series itself diverges.  Each column keeps its own Krylov space and
 * runs until ||b - Z_l x|| <= refine_tol ||b|| (checked on the true residual
 * at the end of a cycle) or max_passes Arnoldi steps in all; restart is the
 * cycle length (0 = 30, at most 64).  The call synchronises the stream once
 * per step (the stopping test), so it cannot be captured into a graph.
 * Statistics: passes = Arnoldi steps the column was active, resid_rel = the
 * true final relative residual, growth = 0, diverged = resid_rel above
 * refine_tol; HM_EDIVERGED is returned then.  On a batched handle a column
 * is one Krylov space over every instance, and ||b|| above (and in
 * resid_rel) is the smallest nonzero ||b_i|| of the column's instances, so
 * that each instance's residual, which is at most the column's, meets
 * refine_tol relative to its own right-hand side.  The request server takes
 * it (the workspace counts against its budget).
 * Workspace: (2 restart + 1) vectors of N x nrhs complex128, kept on the
 * handle. */
/* PS_NESTED: the nested multi-level form of eq. 14-22,
 *   x = (I + X_n)^{-1} ... (I + X_1)^{-1} D^{-1} b,
 * with factors from the leaf level up: X_1 = D^{-1} R_L (near off-diagonal
 * and leaf-level far blocks), X_j = (I + X_{j-1})^{-1} ... (I + X_1)^{-1}
 * D^{-1} F_j for the far blocks F_j of the j-th level above the leaf (the
 * paper's V_2, W_3), down to `level` (levels without far blocks are
 * skipped).  Each inverse is its K-term power series and applying X_j
 * applies the truncated inverses before it, so a solve costs (K + 1)^n - 1
 * level products for n factors (HM_EINVAL above 100,000).  At the leaf level
 * (n = 1) it equals PS_SERIES.  precision selects the block copies of the
 * level products; D^{-1} is FP64.  Statistics: t_ms only.  Single-instance
 * handles only; the request server does not take it. */
enum { PS_SERIES = 0, PS_REFINE = 1, PS_REFINE_FIXED = 2, PS_GMRES = 3, PS_NESTED = 4 };

#define HM_BUILD_HOST_ONLY 0x1u /* build tree, partition and blocks on the host
                                   only: no device memory, for hmat_export /
                                   hmat_info; device calls return HM_ESTATE */
#define HM_BUILD_NO_F32    0x2u /* do not keep FP32 block copies */
#define HM_BUILD_KEEP_HOST 0x4u /* keep the host copy of the blocks after the
                                   upload so that hmat_export works on a
                                   device-built handle */
#define HM_BUILD_NO_HALF   0x8u /* do not build the half-storage data of a
                                   symmetric problem (it serves one right-
                                   hand side: the scaled series and the one-
                                   RHS H-matvec); saves its device memory and
                                   build time on handles for many RHS */

/* ---- problem and options -------------------------------------------------- */
/* Entries of Z (synthetic point-kernel stand-in for the MoM matrix of eq. 5,
 * one unknown per point, e^{-jkR} convention):
 *   surface  Z_ij = h^2 e^{-jkR}/(4 pi R)            i != j,  Z_ii = 2h(1 + 0.1j)
 *   volume   Z_ij = k^2 chi_j h^3 e^{-jkR}/(4 pi R)  i != j,  Z_ii = 1/chi_i + 0.5
 * Coincident points (R < 1e-12) are rejected with HM_EINVAL. */
typedef struct {
  int64_t n;          /* number of unknowns, >= 1                         */
  const double* xyz;  /* host, n x 3 row-major, wavelengths; copied        */
  int32_t kind;       /* HM_SURFACE or HM_VOLUME                           */
  double k;           /* wavenumber                                        */
  double h;           /* spacing (surface) or cell edge (volume)           */
  const double* chi;  /* host, n contrasts (HM_VOLUME), else NULL; copied  */
} hm_problem;

/* Cluster tree (Sec. III): split while a cluster has more than leaf_max
 * points, along the longest bounding-box axis at the median (ties by
 * original index).  Admissibility eq. 7 with eta.  Far blocks: ACA with
 * partial pivoting plus recompression to aca_tol, rank <= max_rank (0 = no
 * cap); only the block with the smaller row offset is compressed and its
 * mirror is the transpose (half H-matrix, Sec. III). */
typedef struct {
  int32_t leaf_max;     /* >= 1 (<= 256)                                    */
  double eta;           /* admissibility parameter, the paper uses 1.0      */
  double aca_tol;       /* relative ACA / recompression tolerance, > 0      */
  int32_t max_rank;     /* 0 = min(m, n)                                    */
  uint32_t flags;       /* HM_BUILD_*                                       */
  int32_t num_threads;  /* host threads for the build, 0 = all             */
  /* optional: called on the building thread as the build advances (phase
   * done, instances built); msg is valid during the call only */
  void (*progress)(const char* msg, void* user);
  void* progress_user;
} hm_build_opts;

typedef struct {
  int32_t K;            /* highest power of the series (K + 1 terms), >= 0 */
  int32_t level;        /* far blocks of level >= level are used; -1 = leaf
                           level only (the paper's runs); levels below the
                           coarsest far level act as the coarsest          */
  int32_t precision;    /* HM_F64 or HM_F32_APPLY                           */
  int32_t kind;         /* PS_SERIES, PS_REFINE, PS_REFINE_FIXED, PS_GMRES,
                           PS_NESTED                                       */
  int32_t max_passes;   /* PS_REFINE: pass limit; PS_REFINE_FIXED: passes;
                           PS_GMRES: Arnoldi step limit                     */
  double refine_tol;    /* PS_REFINE: stop when ||d|| <= tol ||x|| per RHS;
                           PS_GMRES: when ||b - Z_l x|| <= tol ||b||         */
  int32_t restart;      /* PS_GMRES: cycle length, 0 = 30; else ignored     */
} ps_opts;

/* Per right-hand side statistics.  Filling them synchronises the stream. */
typedef struct {
  int32_t passes;       /* refinement passes done (0 for PS_SERIES)         */
  int32_t diverged;     /* 1 if growth > 1 or non-finite values, or (both
                           refinement kinds) last ||d|| > refine_tol ||x||  */
  double resid_rel;     /* refinement: last ||d|| / ||x||; else 0          */
  double growth;        /* ||y_K|| / ||y_0|| of the (last) series           */
  double t_ms;          /* wall time of the whole call (same for all RHS);
                           server tickets: submit to done                  */
  int32_t built;        /* server tickets: 1 if the request's batch had to
                           build its geometry (cold), else 0               */
  int32_t reserved_;
} ps_stats;

#define HM_MAX_LEVELS 32
typedef struct {
  int64_t n;
  int32_t leaf_level;               /* depth L of the deepest leaf           */
  int32_t num_leaves;
  int32_t max_leaf;                 /* largest leaf size                     */
  int32_t min_far_level;            /* coarsest level holding far blocks, or -1 */
  int64_t near_blocks;              /* including the diagonal blocks         */
  int64_t near_offdiag_entries;     /* sum m n over off-diagonal near blocks */
  int64_t diag_entries;             /* sum m^2 over leaves                   */
  int64_t far_blocks[HM_MAX_LEVELS];   /* per level, both orientations      */
  int64_t far_rank_sum[HM_MAX_LEVELS];
  int64_t far_entries[HM_MAX_LEVELS];  /* sum r (m + n)                      */
  int64_t device_bytes;             /* device memory held by the handle     */
  double build_ms;                  /* host build + upload + device LU       */
  /* Entries (complex elements) a product at far level l reads, by level;
   * zero for levels without far blocks when far blocks exist elsewhere:
   *   series_entries  D^{-1}-premultiplied near and far columns (one term)
   *   apply_entries   D, near and far columns of Z_l (one H-matvec)
   *   stageA_entries  W_b of the far blocks of level >= l
   *   coeffs          stage-A coefficients of the far blocks of level >= l */
  int64_t series_entries[HM_MAX_LEVELS];
  int64_t apply_entries[HM_MAX_LEVELS];
  int64_t stageA_entries[HM_MAX_LEVELS];
  int64_t coeffs[HM_MAX_LEVELS];
  int32_t num_instances;            /* 1, or the count of a batched handle  */
  int64_t half_entries[HM_MAX_LEVELS]; /* entries the half-storage
                                        product reads per term: near
                                        blocks (t, s > t) once, far blocks
                                        between two leaves once (U and W),
                                        U and W of the other far blocks per
                                        orientation (0: not symmetric) */
} hm_info;

/* Kernel classes timed by hm_profile_enable. */
enum {
  HM_K_STAGEA = 0,       /* t_b = W_b y_s for far blocks whose row cluster
                            spans several leaves (levels above the leaf level) */
  HM_K_TERM_SERIES = 1,  /* one power-series term: D^{-1}-premultiplied near
                            and far products, in-row low-rank blocks, y and x
                            update (one launch per term)                      */
  HM_K_TERM_APPLY = 2,   /* one H-matvec (hmat_apply, refinement residual)   */
  HM_K_TERM_DINV = 3,    /* y_0 = D^{-1} b                                    */
  HM_K_COUNT = 4
};
typedef struct {
  int64_t launches;
  double total_ms;        /* sum of per-launch durations from HIP events    */
} hm_kernel_time;

typedef struct hm_matrix* hm_matrix_t;

/* ---- H-matrix ------------------------------------------------------------- */

/* Build the H-matrix of `prob` (Sec. III): tree, partition, near fill, ACA
 * with recompression on the host; upload; leaf LU with partial pivoting
 * (eq. 12's near-field inverse) and D^{-1} on the device.  Synchronises
 * `hip_stream` before returning.  *out is set only on success. */
int hmat_build(const hm_problem* prob, const hm_build_opts* opts, void* hip_stream,
               hm_matrix_t* out);

/* Batched build: `count` independent problems (sizes may differ) with the
 * same options, merged into one block-diagonal H-matrix so that one
 * persistent launch per series term serves all of them.  Vectors passed to
 * hmat_apply / ps_solve on the handle hold the instances one after another
 * (instance i at rows off_i .. off_i + n_i - 1, off_i = n_0 + ... + n_{i-1}),
 * each in its own original point order.  Levels of a batched handle count
 * from the top: level -1 (or HM_MAX_LEVELS - 1) selects every instance's
 * leaf-level far blocks, HM_MAX_LEVELS - 1 - d adds the blocks up to d levels
 * above each instance's leaf level.  hmat_info reports levels the same way. */
int hmat_build_batched(const hm_problem* probs, int32_t count, const hm_build_opts* opts,
                       void* hip_stream, hm_matrix_t* out);

/* Structure statistics (host only, no device access). */
int hmat_info(hm_matrix_t h, hm_info* out);

/* y = Z_l x (eq. 6 restricted to far levels >= level), including D, for
 * nrhs right-hand sides.  precision HM_F32_APPLY reads the FP32 block
 * copies.  x_dev and y_dev must not overlap. */
int hmat_apply(hm_matrix_t h, int32_t level, int32_t precision, const void* x_dev,
               int64_t ldx, void* y_dev, int64_t ldy, int32_t nrhs, void* hip_stream);

/* Power-series solve (Sec. IV).  b_dev and x_dev must not overlap.  per_rhs
 * (host, nrhs entries) may be NULL; when given, the call synchronises and
 * fills it.  Returns HM_EDIVERGED (> 0) when stats were requested and some
 * right-hand side grew; x is still written. */
int ps_solve(hm_matrix_t h, const ps_opts* opts, const void* b_dev, int64_t ldb, void* x_dev,
             int64_t ldx, int32_t nrhs, ps_stats* per_rhs, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ps_solve
 * without statistics whose workspace (the [y | t] vectors, their FP32
 * shadows, refinement vectors, split-K partial sums and counters) lives in a
 * static device array of HM_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on each device it runs on until the process ends.  Kinds PS_SERIES
 * and PS_REFINE_FIXED only (else HM_EINVAL); other arguments as ps_solve,
 * same kernels and the same results bit for bit.  A call whose workspace
 * would exceed the array (it grows with nrhs and with N plus the stage-A
 * coefficients of the handle) fails with HM_EINVAL before any device work.
 * The call itself allocates nothing and does not synchronise; the handle's
 * own device data (built by hmat_build) is read as with ps_solve.  Every
 * call on one device shares that device's array: calls that overlap in
 * time on one device (on different streams or from different threads) race
 * and give wrong results; the counters that must start at zero are
 * cleared by each call (a fill kernel, so the call can be captured). */
#define HM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ps_solve_noalloc(hm_matrix_t h, const ps_opts* opts, const void* b_dev, int64_t ldb,
                     void* x_dev, int64_t ldx, int32_t nrhs, void* hip_stream);

/* Write the host-side H-matrix (permutation, blocks, factors) to `path` as
 * (needs HM_BUILD_HOST_ONLY or HM_BUILD_KEEP_HOST, else HM_ESTATE)
 * a sequence of named arrays: u32 name length, name bytes, u32 dtype code
 * (1 int32, 2 int64, 3 float64, 4 complex128), u32 ndim, u64 shape[ndim],
 * raw little-endian data.  For checking the build against an independent
 * implementation. */
int hmat_export(hm_matrix_t h, const char* path);

/* Launch tuning of a device handle.  mm_min_rhs: from this many
 * right-hand sides on, the term and stage-A products of ps_solve and
 * hmat_apply run as matrix-core (MFMA) contractions over tiles of 16, 32 or
 * 64 right-hand sides (FP32 blocks: three real products per complex one;
 * FP64: four); below it, one-RHS-tile streaming kernels run (default 8).
 * term_wgs: persistent workgroups per term launch (the work lists are split
 * evenly over them; default: compute units x resident workgroups per unit).
 * Results do not depend on these values beyond rounding order.  Changing
 * term_wgs or inrow_pct rebuilds the work lists (synchronises the stream); the handle
 * must not be in use on another stream meanwhile.  In hmat_tune a field of
 * 0 keeps its value and -1 restores the default. */
typedef struct {
  int32_t mm_min_rhs;
  int32_t term_wgs;
  int32_t rhs_tile;   /* MFMA right-hand-side tile per workgroup: 16, 32 or
                         64 (0 or -1 in hmat_tune: chosen from nrhs)       */
  int32_t inrow_pct;  /* streaming kernels: cost weight (percent) of a row of
                         a leaf-level low-rank block against a dense panel
                         column in the even split of the work (default 100;
                         changing it rebuilds the work lists)              */
  int32_t half_storage; /* 1 (default): the series, refinement and GMRES
                         of one right-hand side (below mm_min_rhs) run in
                         the scaled basis D = C C^T, S = C^{-1} R C^{-T} on
                         half storage (a surface problem is symmetric; a
                         volume problem Z = A diag(chi) runs on its
                         symmetric A, x = diag(1/chi) x_A):
                         each off-diagonal near block S_ts, s > t, and
                         each far block between two leaves t < s is read
                         once and applied in both orientations
                         (S_st = S_ts^T), and where every far block of the
                         level lies between two leaves the K terms run as
                         one launch; 3: half storage with one launch per
                         term; 2: the D^{-1}-premultiplied panels.
                         With 1 or 3, hmat_apply of one right-hand side
                         on such a problem reads the half storage too,
                         as Z x = C (I + S) C^T x                          */
  int32_t mm_multi;     /* 2 (default): one launch per stage A and per term
                         of the many-RHS series on the matrix cores; 1: the
                         K terms (stage A included) as one persistent
                         launch where the handle allows it (leaves of at
                         most 64 rows, at most 32 right-hand sides,
                         K <= 16), per-instance counters ordering the terms
                         of each batched instance; measured 1.02-1.22x
                         the time of the per-term launches on 16 to 256
                         instances, so the autotuner times both            */
} hm_tuning;
int hmat_tune(hm_matrix_t h, const hm_tuning* t, void* hip_stream);
int hmat_get_tuning(hm_matrix_t h, hm_tuning* out);

/* Autotuner: times ps_solve with opts (series kind) on nrhs zero
 * right-hand sides (vectors the call allocates and frees) for every
 * candidate tuning -- term_wgs in {auto, auto/2, 2 auto, 4 auto} times
 * {streaming kernels with inrow_pct 100/150/200, MFMA kernels with RHS
 * tiles 16/32/64 up to nrhs, each with the K terms in one launch and per
 * term}, and the half-storage kernel where it
 * applies --
 * and keeps the fastest on the handle (median of five timed calls after
 * two warm-ups, HIP events on hip_stream).  When an MFMA candidate wins,
 * mm_min_rhs becomes min(nrhs, 8), so one right-hand side keeps the
 * streaming kernels; when a streaming one wins, nrhs + 1.  best and best_ms (nullable)
 * receive the choice and its time per solve.  Synchronises the stream. */
int hmat_autotune(hm_matrix_t h, const ps_opts* opts, int32_t nrhs, void* hip_stream,
                  hm_tuning* best, double* best_ms);

/* Per-kernel timing for measurement: while enabled, every launch of the
 * classes above is bracketed by HIP events recorded on the launch stream.
 * Enabling (or disabling) resets the counters. */
int hm_profile_enable(hm_matrix_t h, int32_t enable);
/* Synchronise the recorded events and return launches and summed durations
 * per class (out has HM_K_COUNT entries). */
int hm_profile_read(hm_matrix_t h, hm_kernel_time* out);

/* Release the handle and all its device memory (synchronises the device). */
int hmat_free(hm_matrix_t h);

/* ---- request server (continuous batching) ----------------------------------
 * A server owns worker threads, one HIP stream each (max_slots), and a cache
 * of device-resident geometries (trees, LU factors, blocks) under an HBM
 * budget.  ps_submit queues a solve of nrhs (1..64) right-hand sides on the
 * geometry geom_key; the first submit of a key must give its problem and
 * build options (both copied; later submits may pass NULL).  b_host (n x
 * nrhs complex128, column-major, original order) is copied, so the caller
 * may reuse it at once.  A free worker takes the oldest queued request
 * whose geometry is not in use and every later queued request of the same
 * geometry and options up to 64 right-hand sides in all, and solves them as
 * one ps_solve; batches of different geometries run at the same time on
 * different streams, and requests that arrive meanwhile join the next
 * batch of their geometry.  A geometry is built on its first batch and
 * kept; to admit a build, least recently used geometries without queued
 * or running requests are freed until blocks plus workspaces fit the
 * budget (a geometry that cannot fit an idle device fails with HM_ENOMEM).
 * Solve kinds: PS_SERIES, PS_REFINE, PS_REFINE_FIXED and PS_GMRES (whose
 * basis, kept on the geometry, is admitted under the budget the same way);
 * PS_NESTED is refused.
 * Results: ps_poll returns HM_ENOTREADY while the ticket is queued or
 * running.  Once it is done (or failed) it returns the solve's status and
 * copies x (n x nrhs, original order) to x_host and the per-RHS statistics
 * (t_ms = submit-to-done latency) to per_rhs, each when non-null; a poll
 * with x_host or per_rhs given releases the ticket (a later poll of it is
 * HM_EINVAL), a poll with both NULL only reports the state.  Server calls are thread-safe.  hbm_budget_bytes 0
 * means 90% of the device memory free at creation. */
typedef struct hm_server* hm_server_t;
typedef uint64_t hm_ticket_t;
enum { PS_QUEUED = 0, PS_RUNNING = 1, PS_DONE = 2, PS_FAILED = 3 };
typedef struct {
  int64_t budget_bytes, resident_bytes, resident_geometries;
  int64_t builds, evictions;         /* geometry builds (incl. rebuilds)    */
  int64_t batches, batch_rhs;        /* solves issued and their columns     */
  int64_t requests_submitted, requests_done, requests_failed, rhs_done;
  int64_t queued;
  int64_t split_batches;             /* batches solved in pieces of the
                                        existing workspace's width (no room
                                        for a wider one)                   */
} ps_server_stats;
int ps_server_create(size_t hbm_budget_bytes, int32_t max_slots, hm_server_t* out);
int ps_submit(hm_server_t s, uint64_t geom_key, const hm_problem* prob,
              const hm_build_opts* build_opts, const ps_opts* opts, const void* b_host,
              int32_t nrhs, hm_ticket_t* out);
int ps_poll(hm_server_t s, hm_ticket_t ticket, void* x_host, ps_stats* per_rhs, int32_t* state);
int ps_server_info(hm_server_t s, ps_server_stats* out);
/* Waits for running batches, fails queued tickets, frees every geometry. */
int ps_server_destroy(hm_server_t s);

/* ---- errors ----------------------------------------------------------------- */
const char* hm_strerror(int status);
const char* hm_last_error(void);   /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* HMPS_H */
