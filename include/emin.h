/*
 * emin.h -- C ABI of the MI355X (gfx950) EMIN-AMG grid-transfer library for
 * Q2-Q1 (Taylor-Hood) saddle-point systems, after Prokopenko & Tuminaro,
 * "An algebraic multigrid method for Q2-Q1 mixed discretizations of the
 * Navier-Stokes equations" (arXiv:1607.02489).
 *
 * One level of the paper's Alg. 1 (setup_hierarchy, without relaxation) is
 *   emin_pattern  -- Alg. 2 up to the sparsity patterns: aux operators of
 *                    eq. (e:filtering), Alg. 3 coarse pressures, Alg. 4
 *                    mid-points and coarse velocities, patterns N^(p), N^(v),
 *                    and the symbolic Galerkin product;
 *   emin_setup    -- sec. 4.3, eq. (min_problem): the prolongator values by
 *                    constrained CG on trace(P^T M P) from the normalised
 *                    binary pattern;
 *   emin_rap      -- Alg. 1, A_{l+1} = R A P with R = P^T.
 * The coarse operator's patterns live in the pattern handle; its values in
 * caller buffers, so a hierarchy is built by feeding level l's views and
 * values to level l+1.
 *
 * Conventions
 *  - All array pointers are DEVICE pointers unless the comment says host.
 *  - CSR: rowptr int64[nrows+1], col int32[nnz] sorted and unique per row,
 *    val double[nnz].
 *  - The velocity block of the saddle system is I_d (x) Ahat (identical
 *    component blocks, sec. 2); Bdiv holds the divergence block with the
 *    column of component c of velocity node k at c*n_v + k.
 *  - A Dirichlet (eliminated) velocity node is one whose Ahat row has no
 *    nonzero off-diagonal value.
 *  - stream is a hipStream_t (NULL = the default stream).  emin_pattern
 *    synchronises the stream (it reads sizes back); emin_setup and
 *    emin_rap only enqueue work and never synchronise.
 *  - No exception crosses the ABI.  On error the outputs are untouched and
 *    *out stays NULL.  A handle is not thread-safe; distinct handles are
 *    independent.  Calls on one handle must not overlap in time.
 */
#ifndef EMIN_H
#define EMIN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EMIN_OK = 0,
  EMIN_ERR_ARG = 1,         /* NULL pointer, negative size, bad parameter */
  EMIN_ERR_SHAPE = 2,       /* inconsistent dimensions between inputs */
  EMIN_ERR_PATTERN = 3,     /* CSR columns unsorted, duplicated or out of range */
  EMIN_ERR_VALUE = 4,       /* NaN/Inf in values (checked with EMIN_FLAG_VALIDATE) */
  EMIN_ERR_INFEASIBLE = 5,  /* a row cannot meet P W_c = W (empty pattern, W_i != 0) */
  EMIN_ERR_BREAKDOWN = 6,   /* CG met <Z, M Z> <= 0 while <R, R> > 0 */
  EMIN_ERR_BUDGET = 7,      /* request exceeds the device-memory budget */
  EMIN_ERR_DEVICE = 8,      /* HIP runtime error */
  EMIN_ERR_OOM = 9,         /* device allocation failed */
  EMIN_ERR_CAPACITY = 10,   /* a fixed per-row/per-ball capacity was exceeded */
  EMIN_ERR_COLOCATE = 11,   /* a coarse pressure without a co-located coarse velocity */
  EMIN_ERR_CANCELLED = 12   /* a served request cancelled before it started */
} emin_status;

enum { EMIN_PREC_F64 = 0, EMIN_PREC_MIXED = 1 };
enum {
  EMIN_FLAG_ENERGY = 1u,    /* emin_setup: record the energy trace(P^T M P) per step */
  EMIN_FLAG_VALIDATE = 2u,  /* check values for NaN/Inf */
  EMIN_FLAG_AUTOTUNE = 4u,  /* emin_pattern: time candidate schedules of the masked
                               product on this pattern (or reuse the choice made for
                               the same problem shape) and keep the fastest */
  EMIN_FLAG_PATTERN_VALUES = 8u, /* emin_setup: the system's values are still those the
                                    handle's emin_pattern call was given, so the
                                    filtered operators that call formed are reused
                                    instead of being formed again (the caller vouches
                                    for it; nothing checks the values) */
  EMIN_FLAG_ENERGY_ATA = 16u,    /* sec. 4.3, eq. (min_problem): the velocity block's
                                    energy is the A^T A-norm of the filtered operator,
                                    trace(P^T A~^T A~ P), the norm the section names for
                                    non-symmetric operators, instead of the norm of its
                                    symmetric part; the velocity graph and the pressure
                                    block are unchanged.  emin_pattern forms A~^T A~;
                                    emin_setup must pass the same flag (EMIN_ERR_ARG
                                    otherwise).  EMIN_VIEW_MV is then A~^T A~. */
  EMIN_FLAG_STAGED_PRODUCT = 32u, /* emin_pattern / emin_setup_with_pattern: the masked
                                    product groups rows into tiles by the cells of a
                                    grid over their coordinates (emin_pattern; blocks
                                    of consecutive rows in emin_setup_with_pattern),
                                    stages each tile's Z rows in LDS (coalesced runs)
                                    and sums from LDS, instead of gathering Z from
                                    device memory row by row; rows of tiles that do not
                                    fit keep the gathering kernel.  Each output is the
                                    same sum in another fixed order (partials over every
                                    eighth entry, added in a fixed tree): deterministic,
                                    equal to the gathering kernel's up to rounding */
  EMIN_FLAG_GMRES = 64u,         /* sec. 4.3 names a constrained CG or GMRES: the velocity
                                    block's EMIN runs `iters` steps of GMRES on the
                                    projected masked system Pi mask_N(A~ P) = 0 of the
                                    filtered, non-symmetric operator A~ itself, from the
                                    same start P0 (the iterate minimises the projected
                                    residual over the Krylov space); the report's rho_v
                                    then holds the squared residual norms and energy_v
                                    stays 0.  Not with EMIN_FLAG_ENERGY_ATA; emin_setup
                                    must pass the same flag.  EMIN_VIEW_MV is then A~. */
  EMIN_FLAG_PETROV_GALERKIN = 128u /* sec. 4.3, last paragraph: the restriction is not P^T.
                                    emin_pattern also prepares a second minimisation for
                                    R_v^T on the velocity pattern, in the A A^T-norm of
                                    the filtered block (with EMIN_FLAG_GMRES: the GMRES
                                    form on A~^T); emin_setup_pg computes it and
                                    emin_rap_pg the Petrov-Galerkin coarse blocks.  R_p
                                    stays P_p^T (its operator is symmetric). */
};
#define EMIN_MAX_ITERS 32

typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t *rowptr;
  const int32_t *col;
  const double *val;
} emin_csr_t;

/* One level's saddle system (sec. 2): [I_d (x) Ahat, Bdiv^T; Bdiv, 0]. */
typedef struct {
  int32_t dim;              /* spatial dimension d: 2 or 3 */
  emin_csr_t Ahat;          /* n_v x n_v scalar velocity block (Stokes or Oseen) */
  emin_csr_t Bdiv;          /* n_p x d*n_v divergence block */
  const double *xv;         /* n_v*d velocity node coordinates (row-major) */
  const int32_t *p2v;       /* n_p: velocity node co-located with each pressure */
  const double *Wv;         /* n_v near-nullspace mode or NULL: 1 off the Dirichlet set */
  const double *Wp;         /* n_p near-nullspace mode or NULL: all ones */
  const double *Gt;         /* the gradient (1,2) block's transpose, its values on Bdiv's
                               pattern, or NULL when it is Bdiv^T (a fine level; every
                               level with R = P^T).  Read by emin_rap_pg only. */
} emin_system_t;

/* Parameters (sec. 6 uses tau1 = 0.06 and tau2 = sqrt(1.5e-3)). */
typedef struct {
  double tau1_v;            /* drop tolerance of eq. (e:filtering), velocity block */
  double tau1_p;            /* drop tolerance of eq. (e:filtering), B B^T */
  double tau2_sq;           /* tau2^2 of Alg. 4's closeness test */
  int32_t iters;            /* EMIN CG steps, 0..EMIN_MAX_ITERS */
  int32_t precision;        /* EMIN_PREC_F64, or EMIN_PREC_MIXED: FP32 masked
                               products and RAP, FP64 projection and scalars */
  uint32_t flags;           /* EMIN_FLAG_* */
} emin_params_t;

/* Sizes of one level (host struct). */
typedef struct {
  int64_t n_v, n_p;         /* fine velocity nodes, fine pressures */
  int64_t n_vc, n_pc;       /* coarse velocity nodes, coarse pressures */
  int64_t n_cp_alg3;        /* C^(p) points chosen by Alg. 3 */
  int64_t n_cp_extra;       /* C^(p) points added by the extra distance-3 pass */
  int64_t n_mid;            /* mid-points added by Alg. 4 */
  int64_t n_cv_extra;       /* C^(v) points added for uncovered velocity nodes */
  int64_t nnz_Pv, nnz_Pp;   /* pattern sizes of the scalar velocity and pressure P */
  int64_t nnz_Mv, nnz_Mp;   /* energy operators */
  int64_t nnz_Ac, nnz_Bc;   /* coarse scalar velocity block and coarse divergence */
  int64_t device_bytes;     /* device memory held by the handle */
  int64_t sched_v, sched_p; /* masked-product schedule of each block: bit 0 intersection
                               maps used, bit 1 lanes per row doubled, bit 2 XCD split by
                               row class, bit 3 blocks of all classes in row order with
                               one contiguous eighth per XCD (neither: one contiguous
                               eighth of the class-major grid per XCD); bits 4-5: 0
                               default, 1 autotuned on this pattern, 2 reused from an
                               earlier tuning of the same shape; bit 6: blocks of rows
                               staged in LDS (the other rows follow bits 0-3); bit 7:
                               map rows gather 16 M entries per batch instead of 4 */
} emin_sizes_t;

/* Device-resident report of emin_setup (read it with emin_sync_report). */
typedef struct {
  int32_t status;           /* emin_status of the numeric phase */
  int32_t its_v, its_p;     /* CG steps taken per block */
  int32_t reserved;
  double energy_v[EMIN_MAX_ITERS + 1], energy_p[EMIN_MAX_ITERS + 1];
  double rho_v[EMIN_MAX_ITERS + 1], rho_p[EMIN_MAX_ITERS + 1];
  double gamma_v[EMIN_MAX_ITERS], gamma_p[EMIN_MAX_ITERS];
  /* the Petrov-Galerkin restriction's minimisation (emin_setup_pg) */
  int32_t its_r, reserved2;
  double energy_r[EMIN_MAX_ITERS + 1], rho_r[EMIN_MAX_ITERS + 1], gamma_r[EMIN_MAX_ITERS];
} emin_report_t;

/* Read-only device views held by a pattern handle (valid until destroy). */
enum {
  EMIN_VIEW_PV = 0,    /* CSR pattern of the scalar velocity P (n_v x n_vc) */
  EMIN_VIEW_PP = 1,    /* CSR pattern of P^(p) (n_p x n_pc) */
  EMIN_VIEW_AC = 2,    /* CSR pattern of the coarse scalar velocity block */
  EMIN_VIEW_BC = 3,    /* CSR pattern of the coarse divergence block */
  EMIN_VIEW_MV = 4,    /* CSR energy operator, velocity (values after emin_setup) */
  EMIN_VIEW_MP = 5,    /* CSR energy operator, pressure (values after emin_setup) */
  EMIN_VIEW_S = 6,     /* CSR of the S sets: fine C^(p) within distance 3, sorted */
  EMIN_VIEW_ORDER = 7, /* int32[n_cp_alg3 + n_cp_extra]: C^(p) in selection order */
  EMIN_VIEW_CP = 8,    /* int32[n_pc]: C^(p), ascending fine index */
  EMIN_VIEW_CBAR = 9,  /* uint8[n_p]: 1 on C-bar^(p) (C^(p) and mid-points) */
  EMIN_VIEW_CV = 10,   /* int32[n_vc]: C^(v), ascending fine index */
  EMIN_VIEW_XVC = 11,  /* double[n_vc*d]: coarse velocity coordinates */
  EMIN_VIEW_P2VC = 12, /* int32[n_pc]: coarse co-location map */
  EMIN_VIEW_KEEPV = 13,/* uint8[nnz(Ahat)]: kept entries of the velocity filter */
  EMIN_VIEW_KEEPP = 14,/* uint8[nnz(B B^T)]: kept entries of the pressure filter */
  EMIN_VIEW_DIR = 15   /* uint8[n_v]: Dirichlet velocity nodes */
};
typedef struct {
  int64_t n;                /* rows (CSR) or elements (arrays) */
  int64_t ncols;            /* CSR columns (0 for arrays) */
  int64_t nnz;              /* CSR nonzeros (0 for arrays) */
  const int64_t *rowptr;    /* CSR only */
  const int32_t *col;       /* CSR only */
  const double *val;        /* CSR values when present, else NULL */
  const void *data;         /* arrays */
} emin_view_t;

typedef struct emin_pattern_s emin_pattern_t;

/* Device memory supplied by the caller (e.g. a framework's caching
 * allocator).  alloc(bytes, ctx) returns device memory of the current device,
 * at least 256-byte aligned, or NULL; free(ptr, ctx) takes back a block alloc
 * returned.  Both are called from the thread that calls the library. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *ctx;
} emin_allocator_t;

/* Alg. 2 up to the patterns, plus the symbolic RAP and the coarse
 * descriptors (coordinates by injection, co-location map).  Borrows sys for
 * the call; the handle owns its device memory (hipMalloc) until destroyed.
 * Errors: ARG/SHAPE/PATTERN on bad inputs, CAPACITY, COLOCATE, DEVICE, OOM. */
emin_status emin_pattern(const emin_system_t *sys, const emin_params_t *prm, void *stream,
                         emin_pattern_t **out);
/* emin_pattern with every device block of the handle (the pattern phase's
 * arrays, the EMIN workspace, the RAP plans) taken from *alloc and given
 * back through it by emin_pattern_destroy, once the work the library queued
 * on the block has completed (or when the call fails, after the stream has
 * drained).  alloc = NULL: the library's own memory, as
 * emin_pattern.  A block that is not 256-byte aligned is given back and the
 * call fails with EMIN_ERR_ARG; alloc returning NULL fails it with
 * EMIN_ERR_OOM.  The allocator must outlive the handle. */
emin_status emin_pattern_alloc(const emin_system_t *sys, const emin_params_t *prm,
                               const emin_allocator_t *alloc, void *stream,
                               emin_pattern_t **out);

/* emin_pattern with the coarse pressures C^(p) given instead of chosen by
 * Alg. 3 and the extra distance-3 pass (sec. 4.1): cp holds ncp ascending,
 * distinct fine pressure indices (device memory, borrowed for the call).
 * Everything after the coarse pressures is as in emin_pattern: the S sets
 * (every given C point within graph distance 3 of a vertex, read off the
 * distance-4 balls), Alg. 4's mid-points (sec. 4.2), the velocity pattern,
 * the symbolic Galerkin product and the coarse descriptors.  For a perfect
 * distance-4 coarsening of a uniform mesh, sec. 4.2 fixes C-bar as the
 * spacing-2 pressure lattice, which this call lets a test check on the
 * device.  EMIN_VIEW_ORDER lists the given points.  Errors: as emin_pattern,
 * plus ARG for ncp < 0 or a NULL list, SHAPE for ncp > n_p, PATTERN for an
 * unsorted, repeated or out-of-range list. */
emin_status emin_pattern_with_cpoints(const emin_system_t *sys, const emin_params_t *prm,
                                      const int32_t *cp, int64_t ncp, void *stream,
                                      emin_pattern_t **out);

/* Host copy of the level sizes. */
emin_status emin_pattern_info(const emin_pattern_t *h, emin_sizes_t *out);

/* Device view of one of the handle's arrays (EMIN_VIEW_*). */
emin_status emin_pattern_view(const emin_pattern_t *h, int32_t what, emin_view_t *out);

/* sec. 4.3: energy operators on the stored drop masks, then P0 and `iters`
 * constrained CG steps per block.  sys must have the structure given to
 * emin_pattern (values may differ: successive Picard linearisations).
 * Pv_vals (nnz_Pv) and Pp_vals (nnz_Pp) are caller-allocated outputs.
 * report may be NULL; device-side INFEASIBLE/BREAKDOWN land in report->status.
 * Asynchronous on stream; uses workspace held by the handle. */
emin_status emin_setup(emin_pattern_t *h, const emin_system_t *sys, const emin_params_t *prm,
                       double *Pv_vals, double *Pp_vals, void *stream, emin_report_t *report);

/* sec. 4.3, eq. (min_problem) on one block with every ingredient given:
 * minimise trace(P^T M P) over P with the pattern N and P W_c = W, by
 * `iters` constrained CG steps from P0 = W_i W_c / sum_{N_i} W_c^2 (the same
 * kernels emin_setup runs on each block).
 *   M        n x n CSR energy operator (symmetric positive semi-definite on
 *            the feasible updates), borrowed;
 *   N_rowptr int64[n+1], N_col int32[nnz_N]: the pattern, columns sorted in
 *            [0, ncoarse), at most 64 per row;
 *   cid      int32[n]: the coarse column of a C row (its pattern must be
 *            exactly that column; the row is held at 1), -1 for other rows;
 *   W        double[n], Wc double[ncoarse]: the near-nullspace mode and its
 *            coarse restriction;
 *   P_vals   double[nnz_N] out (caller-allocated);
 *   precision EMIN_PREC_F64 or EMIN_PREC_MIXED; flags: EMIN_FLAG_ENERGY
 *            records the energy, EMIN_FLAG_VALIDATE checks M's values;
 *   report   device emin_report_t or NULL; the block's trace is in the _v
 *            fields, INFEASIBLE (an F row with an empty pattern and W_i != 0)
 *            and BREAKDOWN (<Z, M Z> <= 0 while <R, R> > 0) in status.
 * Allocates its workspace for the call and synchronises the stream before
 * returning.  Errors: ARG, SHAPE, PATTERN (malformed N, or a C row whose
 * pattern is not its own column), VALUE, CAPACITY (a pattern row > 64). */
emin_status emin_setup_with_pattern(const emin_csr_t *M, const int64_t *N_rowptr,
                                    const int32_t *N_col, int64_t ncoarse, int64_t nnz_N,
                                    const int32_t *cid, const double *W, const double *Wc,
                                    int32_t iters, int32_t precision, uint32_t flags,
                                    double *P_vals, void *stream, emin_report_t *report);

/* emin_setup_with_pattern for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments, the same kernels and the same results,
 * with the workspace taken from a fixed 64 MiB device array the library
 * holds on every GPU it runs on (until the process ends) instead of
 * allocated.  No hipMalloc, hipFree or allocating library call is made.
 * Problems whose workspace bound exceeds 64 MiB (about 1e5 rows with 1e6
 * pattern entries and 2e6 operator entries) are rejected with
 * EMIN_ERR_CAPACITY before any work is queued; EMIN_FLAG_STAGED_PRODUCT is
 * rejected with EMIN_ERR_ARG.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (several host threads or streams) race, so
 * the caller serialises them.  Synchronises the stream before returning. */
emin_status emin_setup_with_pattern_noalloc(const emin_csr_t *M, const int64_t *N_rowptr,
                                            const int32_t *N_col, int64_t ncoarse, int64_t nnz_N,
                                            const int32_t *cid, const double *W, const double *Wc,
                                            int32_t iters, int32_t precision, uint32_t flags,
                                            double *P_vals, void *stream, emin_report_t *report);

/* Alg. 1 Galerkin product with R = P^T on the unfiltered operator:
 * Ac = Pv^T Ahat Pv (nnz_Ac values) and Bc = Pp^T Bdiv (I_d (x) Pv)
 * (nnz_Bc values), written into caller buffers on the handle's coarse
 * patterns.  precision EMIN_PREC_MIXED computes the products from FP32
 * copies with FP32 accumulation (results stored as FP64).  Asynchronous on
 * stream (the first mixed call on a handle allocates its FP32 buffers). */
emin_status emin_rap(emin_pattern_t *h, const emin_system_t *sys, const double *Pv_vals,
                     const double *Pp_vals, double *Ac_vals, double *Bc_vals, int32_t precision,
                     void *stream);

/* sec. 4.3, last paragraph (needs EMIN_FLAG_PETROV_GALERKIN at emin_pattern):
 * emin_setup's work plus R_v^T (nnz_Pv values on the velocity pattern,
 * caller-allocated) from the second minimisation, whose trace goes to the
 * report's _r fields.  Asynchronous on stream. */
emin_status emin_setup_pg(emin_pattern_t *h, const emin_system_t *sys, const emin_params_t *prm,
                          double *Pv_vals, double *Pp_vals, double *Rvt_vals, void *stream,
                          emin_report_t *report);

/* Petrov-Galerkin coarse blocks with R_v = Rvt^T and R_p = P_p^T (FP64):
 * Ac = R_v Ahat P_v (nnz_Ac), Bc = P_p^T Bdiv (I_d (x) P_v) (nnz_Bc, the
 * divergence block), and the gradient block's transpose
 * Gct = P_p^T G^T (I_d (x) Rvt) on Bc's pattern (nnz_Bc), G^T being sys->Gt
 * (or Bdiv when NULL).  The next level takes Ac, Bc and Gct (as its Gt).
 * Asynchronous on stream. */
emin_status emin_rap_pg(emin_pattern_t *h, const emin_system_t *sys, const double *Pv_vals,
                        const double *Pp_vals, const double *Rvt_vals, double *Ac_vals,
                        double *Bc_vals, double *Gct_vals, void *stream);

/* Synchronises stream, copies the report to host memory and returns its status. */
emin_status emin_sync_report(const emin_report_t *report, void *stream, emin_report_t *host);

/* Copies bytes from device to host memory (synchronous on stream). */
emin_status emin_memcpy_d2h(void *dst_host, const void *src_dev, size_t bytes, void *stream);

/* Releases the handle.  Its device memory returns to a process-wide cache of
 * chunks that later allocations on the same device reuse (no hipFree, so no
 * device-wide wait).  Work that this library's calls queued on the handle is
 * tracked: its chunks are handed out again only after the last such work has
 * completed.  Two cases stay the caller's to finish before the call: its own
 * work that reads the handle's arrays (emin_pattern_view), and replays of a
 * graph captured from the handle's calls.  NULL-safe. */
void emin_pattern_destroy(emin_pattern_t *h);
/* Frees the cached device chunks (after the work last queued on each has
 * completed); returns the bytes released. */
int64_t emin_release_cached(void);

/* Autotuner bookkeeping (process-wide): out[0] shapes tuned by timing,
 * out[1] patterns that reused a tuned shape, out[2] candidate schedules timed,
 * out[3] entries in the table.  emin_autotune_reset() empties the table. */
emin_status emin_autotune_stats(int64_t *out4);
emin_status emin_autotune_reset(void);

const char *emin_status_string(emin_status s);
const char *emin_version(void);
/* Human-readable detail of the last error returned on the calling thread. */
const char *emin_last_error(void);

/* ------------------------------------------------------------------------
 * Whole hierarchies (Alg. 1 without relaxation)
 * ------------------------------------------------------------------------ */
typedef struct emin_hierarchy_s emin_hierarchy_t;

/* Builds levels 0..nlevels-1 (at most nlevels-1 transfers) by emin_pattern,
 * emin_setup and emin_rap per level, stopping before a level with at most
 * min_dofs dofs.  Level 0's arrays are borrowed (they must stay valid while
 * the hierarchy is re-set up); coarse levels are owned.  Synchronises the
 * stream between levels (emin_pattern reads sizes back). */
emin_status emin_hierarchy_build(const emin_system_t *sys, const emin_params_t *prm,
                                 int32_t nlevels, int64_t min_dofs, void *stream,
                                 emin_hierarchy_t **out);
/* Numeric phases only (emin_setup + emin_rap on every level) for new values
 * of the level-0 system with unchanged structure; asynchronous. */
emin_status emin_hierarchy_resetup(emin_hierarchy_t *h, const emin_system_t *sys, void *stream);
/* Number of transfers built; per_level (host, cap entries) gets the sizes. */
emin_status emin_hierarchy_info(const emin_hierarchy_t *h, int32_t *ntransfers,
                                emin_sizes_t *per_level, int32_t cap);
/* Borrowed device pointers of one transfer level (any output may be NULL). */
emin_status emin_hierarchy_level(const emin_hierarchy_t *h, int32_t level, emin_pattern_t **pat,
                                 const double **Pv, const double **Pp, const double **Ac,
                                 const double **Bc, const emin_report_t **report);
/* Device memory held by the hierarchy and its pattern handles (bytes). */
int64_t emin_hierarchy_device_bytes(const emin_hierarchy_t *h);
/* Same contract as emin_pattern_destroy. */
void emin_hierarchy_destroy(emin_hierarchy_t *h);

/* Batched form: builds count hierarchies concurrently, one host thread and
 * one default-priority HIP stream per concurrent build (at most
 * max_parallel).  out receives count handles; on error all are released. */
emin_status emin_hierarchy_build_batch(const emin_system_t *const *systems, int32_t count,
                                       const emin_params_t *prm, int32_t nlevels,
                                       int64_t min_dofs, int32_t max_parallel,
                                       emin_hierarchy_t **out);
/* Captures the numeric phases of every level of every hierarchy (one
 * branch per hierarchy, forked from and joined to stream) into one hipGraph;
 * emin_batch_run replays it as a single launch.  systems[i] is hierarchy i's
 * level-0 system (borrowed).  The capture contains kernels only. */
typedef struct emin_batch_s emin_batch_t;
emin_status emin_batch_create(emin_hierarchy_t *const *hs, const emin_system_t *const *systems,
                              int32_t count, void *stream, emin_batch_t **out);
emin_status emin_batch_run(emin_batch_t *b, void *stream);
void emin_batch_destroy(emin_batch_t *b);

/* Serving: requests are admitted in arrival order when one of max_slots
 * workers is free and their device-memory estimate fits budget_bytes; each
 * worker builds on its own stream, so admitted requests overlap on the GPU.
 * A request's arrays are borrowed until it completes; its hierarchy stays on
 * the device until released.  submit returns EMIN_ERR_BUDGET for a request
 * larger than the whole budget. */
typedef struct emin_server_s emin_server_t;
emin_status emin_server_create(int64_t budget_bytes, int32_t max_slots, emin_server_t **out);
emin_status emin_server_submit(emin_server_t *srv, const emin_system_t *sys,
                               const emin_params_t *prm, int32_t nlevels, int64_t min_dofs,
                               int64_t *ticket);
emin_status emin_server_poll(emin_server_t *srv, int64_t ticket, int32_t *done);
/* Blocks until the request completes; returns its build status. queue_ms =
 * submit to start, run_ms = start to completion (host clock). */
emin_status emin_server_wait(emin_server_t *srv, int64_t ticket, emin_hierarchy_t **result,
                             double *queue_ms, double *run_ms);
/* Cancels a request that has not started: it leaves the queue, never runs,
 * and its ticket completes with EMIN_ERR_CANCELLED (wait returns it; release
 * frees the ticket).  *cancelled = 1 then, 0 for a request already running
 * or done (unchanged).  Unknown ticket: EMIN_ERR_ARG. */
emin_status emin_server_cancel(emin_server_t *srv, int64_t ticket, int32_t *cancelled);
emin_status emin_server_release(emin_server_t *srv, int64_t ticket);
emin_status emin_server_stats(emin_server_t *srv, int64_t *in_use, int32_t *queued,
                              int32_t *running);
void emin_server_destroy(emin_server_t *srv);

/* ------------------------------------------------------------------------
 * Solve phase (sec. 5.2, sec. 6): Braess-Sarazin relaxation, V-cycle, GMRES
 * ------------------------------------------------------------------------ */
typedef struct emin_solver_s emin_solver_t;

/* Multigrid solver on a hierarchy built from sys (level 0's arrays are
 * borrowed for the solver's lifetime; coarse operators and transfers are the
 * hierarchy's, which must outlive the solver).  Vectors are x = (u, p), u
 * component-blocked (dim blocks of n_v), p of n_p.  Each level gets the
 * Braess-Sarazin relaxation of eq. (bs): D = diag(sum_j |a_ij|) of the scalar
 * velocity block (sec. 5.2), the Schur complement S = B D^-1 B^T formed
 * explicitly, gs_sweeps forward Gauss-Seidel sweeps on it from zero, and the
 * relaxation parameter omega (sec. 6 uses 5 sweeps and 0.666).  The V-cycle
 * runs nu steps before and after the coarse correction with R = P^T and
 * coarse_steps steps on the coarsest level (the paper uses Vanka there; see
 * the design notes).  Synchronous.  Errors: ARG, SHAPE, OOM, DEVICE. */
emin_status emin_solver_create(const emin_system_t *sys, const emin_hierarchy_t *h, int32_t nu,
                               double omega, int32_t gs_sweeps, int32_t coarse_steps,
                               void *stream, emin_solver_t **out);
/* Vector length of a level and the number of Gauss-Seidel dependency levels
 * of its Schur complement (either may be NULL). */
emin_status emin_solver_info(const emin_solver_t *s, int32_t level, int64_t *n,
                             int32_t *gs_levels);
/* One Braess-Sarazin step x <- x + [D/omega, B^T; B, 0]^-1 (f - K x) on a
 * level (device vectors of that level's length); stream-ordered. */
emin_status emin_solver_bs_step(emin_solver_t *s, int32_t level, double *x, const double *f,
                                void *stream);
/* x = V-cycle applied to f on level 0, from x = 0; stream-ordered. */
emin_status emin_solver_vcycle(emin_solver_t *s, const double *f, double *x, void *stream);
/* GMRES from x = 0 preconditioned on the right by the V-cycle, without
 * restart, until the residual estimate is at most rtol ||f|| or maxit steps;
 * *its and *relres (host) receive the steps taken and the final relative
 * residual estimate.  Synchronous. */
emin_status emin_solver_gmres(emin_solver_t *s, const double *f, double *x, double rtol,
                              int32_t maxit, int32_t *its, double *relres, void *stream);
void emin_solver_destroy(emin_solver_t *s);

/* ------------------------------------------------------------------------
 * Inf-sup diagnostic (sec. 6.1, Table 3)
 * ------------------------------------------------------------------------ */
typedef struct emin_matrix_s emin_matrix_t;

/* C = P^T M P in device memory (the projection of a mass matrix to the next
 * level with the level's transfer, sec. 6.1): M square n x n, P n x nc with
 * values (e.g. the velocity pattern view with emin_setup's values).  The
 * structural pattern; sums in ascending order.  Synchronous; *out owns C. */
emin_status emin_galerkin(const emin_csr_t *M, const emin_csr_t *P, void *stream,
                          emin_matrix_t **out);
/* Borrowed device view of the matrix (valid until destroy). */
emin_status emin_matrix_view(const emin_matrix_t *m, emin_csr_t *out);
void emin_matrix_destroy(emin_matrix_t *m);

/* sec. 6.1: the smallest non-zero singular value of
 * B~ = lump(|M_p|)^(-1/2) B lump(|M_v|)^(-1/2), lump(|M|) being the diagonal
 * of row sums of |M| and M_v acting on each of the dim velocity components
 * (B is n_p x dim*n_v, component-blocked columns; M_v n_v x n_v; M_p
 * n_p x n_p).  `steps` Lanczos steps with full re-orthogonalisation on
 * B~ B~^T (at most n_p; n_p steps give its eigenvalues); singular values
 * below rel * sigma_max count as zero (nzero of them, e.g. the hydrostatic
 * pressure of an enclosed flow).  A null vector D_p^(1/2) 1 (B^T 1 = 0) is
 * locked first and counted in nzero, so Lanczos runs on its complement.
 * resid (optional) receives the Lanczos residual norm of sigma_min^2's Ritz
 * vector: some eigenvalue of B~ B~^T lies within resid of sigma_min^2, and a
 * resid small against the gap to the next Ritz value says sigma_min has
 * converged (the smallest Ritz value approaches from above as steps grow).
 * Synchronous; results in host memory.  Errors: ARG, SHAPE, PATTERN, VALUE. */
emin_status emin_infsup(const emin_csr_t *B, const emin_csr_t *Mv, const emin_csr_t *Mp,
                        int32_t dim, int32_t steps, double rel, double *sigma_min,
                        double *resid, int32_t *nzero, int32_t *steps_done, void *stream);

/* Kernel-class profiling with HIP events recorded on the launch stream
 * around each instrumented kernel.  Disabled by default.  collect
 * synchronises on the recorded events, sums launches / device time (ms) /
 * algorithmic bytes and flops per class into out[0..nkinds) (host array),
 * and clears the records. */
enum {
  EMIN_PROF_SPMM = 0,       /* masked product Q = mask_N(M Z) */
  EMIN_PROF_UPDATE = 1,     /* projection + CG update */
  EMIN_PROF_SPGEMM = 2,     /* numeric sparse products (B B^T, RAP) */
  EMIN_PROF_ALG3 = 3,       /* Alg. 3 greedy + extra points */
  EMIN_PROF_ALG4 = 4,       /* Alg. 4 mid-points */
  EMIN_PROF_VPAT = 5,       /* velocity pattern */
  EMIN_PROF_N = 8,
  EMIN_PROF_ONLY = 1 << 30  /* emin_profile_enable(EMIN_PROF_ONLY | (1 << kind) | ...):
                               time only the kinds named; any other nonzero value times
                               all kinds, 0 none */
};
typedef struct {
  int64_t launches;
  double total_ms;
  double bytes;
  double flops;
} emin_kstat_t;
emin_status emin_profile_enable(int enable);
emin_status emin_profile_collect(emin_kstat_t *out, int32_t nkinds);
/* The same records one launch at a time, in launch order (kind, device time
 * in ms, algorithmic bytes and flops): the first cap go to out (host array),
 * *n receives the count; the records are cleared as by collect. */
typedef struct {
  int32_t kind;
  int32_t reserved;
  double ms;
  double bytes;
  double flops;
} emin_klaunch_t;
emin_status emin_profile_launches(emin_klaunch_t *out, int32_t cap, int32_t *n);

/* Test hook: out_sqrt[i] = sqrt(x[i]), out_rcp[i] = 1/x[i] computed by the
 * device exactly as the coarsening kernels compute them (IEEE-rounded, no
 * contraction), so a test can compare them bitwise with the host's.  n
 * elements, device arrays, asynchronous on stream. */
emin_status emin_fp_probe(const double *x, double *out_sqrt, double *out_rcp, int64_t n,
                          void *stream);

#ifdef __cplusplus
}
#endif
#endif
