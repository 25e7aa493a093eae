/*
 * Plain FP64 CPU oracle for the EMIN-AMG Q2-Q1 grid-transfer setup
 * (Prokopenko & Tuminaro, "An algebraic multigrid method for Q2-Q1 mixed
 * discretizations of the Navier-Stokes equations", arXiv:1607.02489).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the parity reference for the
 * HIP path.  It shares no code, header or table with the product library;
 * only the test suite, the benchmark's CPU-baseline leg and the smoke check
 * may load it.
 *
 * Everything is single-threaded, FP64, loops in ascending index order, each
 * product and sum rounded separately (built with -ffp-contract=off).
 * Every function allocates its outputs with malloc; release them with
 * orc_free().  Status codes mirror the product library's numbering.
 */
#ifndef EMIN_ORACLE_H
#define EMIN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_SHAPE = 2, ORC_ERR_PATTERN = 3,
  ORC_ERR_VALUE = 4, ORC_ERR_INFEASIBLE = 5, ORC_ERR_BREAKDOWN = 6
};

typedef struct {
  int64_t nrows, ncols;
  int64_t *rowptr;   /* nrows+1 */
  int32_t *col;      /* nnz, sorted unique per row */
  double *val;       /* nnz (may be NULL for a pattern) */
} orc_csr;

void orc_free(void *p);
void orc_csr_free(orc_csr *a);

/* C = A*B, structural pattern, c_ij = sum over k ascending of a_ik*b_kj. */
int orc_spgemm(const orc_csr *A, const orc_csr *B, orc_csr *C);
/* At = A^T (rows of At in ascending original-row order). */
int orc_transpose(const orc_csr *A, orc_csr *At);
/* Drop/lump filter of eq. (e:filtering): keep off-diagonal a_ij iff
 * a_ij^2 > tau1^2 |a_ii a_jj|; dropped values are added to a_ii in
 * ascending j.  keep (nnz(A) bytes, may be NULL) receives the mask. */
int orc_filter(const orc_csr *A, double tau1, orc_csr *At, uint8_t *keep);
/* M = (A + A^T)/2 on the union pattern. */
int orc_symmetrize(const orc_csr *A, orc_csr *M);
/* Dirichlet rows: 1 iff every stored off-diagonal of row i equals 0.0. */
int orc_dirichlet(const orc_csr *A, uint8_t *dir);

/* Alg. 3 (find_coarse_pressures) + find_extra_dist3_Cpoints.
 * G: graph (off-diagonal structure; values ignored).  x: n*dim coords.
 * Out: is_c[n] (1 = C, 0 = F); S (CSR, per-vertex sorted fine C indices
 * within graph distance 3, sdist = those distances); order = C points in
 * selection order (n_alg3 from Alg. 3, then extras in conversion order). */
int orc_coarsen_pressure(const orc_csr *G, const double *x, int dim,
                         uint8_t *is_c, orc_csr *S, int32_t **sdist,
                         int32_t **order, int64_t *n_c, int64_t *n_alg3);

/* S sets (C within graph distance 3, sorted, with distances) for a given
 * C^(p) flag array; order = the C points ascending. */
int orc_sets_from_cpoints(const orc_csr *G, const uint8_t *is_c, orc_csr *S, int32_t **sdist,
                          int32_t **order, int64_t *n_c);

/* Alg. 4 (find_velocity_Cpoints) mid-point pass. cbar[n] in/out:
 * on entry the C^(p) flags, on exit C-bar^(p). */
int orc_midpoints(const orc_csr *S, const uint8_t *is_c, const double *x,
                  int dim, double tau2_sq, uint8_t *cbar, int64_t *n_added);

/* Velocity coarse points + pattern: cv[n] in/out (entry: co-located
 * mid-point flags; exit: final C^(v) incl. extra points).  Pattern N (CSR,
 * cols = coarse velocity indices) from C^(v) within graph distance 3. */
int orc_velocity_pattern(const orc_csr *G, const uint8_t *dir, uint8_t *cv,
                         orc_csr *N, int64_t *n_extra);

/* Pattern from S sets: C rows {self}, F rows sorted coarse indices of S. */
int orc_pressure_pattern(const orc_csr *S, const uint8_t *is_c, orc_csr *N);

/* EMIN-AMG constrained CG (eq. min_problem): P on pattern N (P->val out),
 * cidx[i] = coarse index of a C row or -1; W[n], Wc[nc] single modes.
 * energy[iters+1], rho[iters+1], gamma[iters] (may be NULL). */
int orc_emin(const orc_csr *M, orc_csr *P, const int32_t *cidx,
             const double *W, const double *Wc, int iters,
             double *energy, double *rho, double *gamma, int *its_done);

/* GMRES form of the same constrained problem for a non-symmetric operator
 * K: k steps of GMRES on Pi mask_N(K P) = 0 from P0; res[iters+1] (may be
 * NULL) receives the squared residual norms. */
int orc_emin_gmres(const orc_csr *K, orc_csr *P, const int32_t *cidx,
                   const double *W, const double *Wc, int iters, double *res, int *its_done);

/* Galerkin product: Ac = Pv^T Ahat Pv, Bc = Pp^T Bdiv (I_d (x) Pv). */
int orc_rap(const orc_csr *Ahat, const orc_csr *Bdiv, int dim,
            const orc_csr *Pv, const orc_csr *Pp, orc_csr *Ac, orc_csr *Bc);

/* One whole level (Alg. 2 + EMIN + RAP + coarse descriptors). */
typedef struct {
  int status;
  int dim;
  /* aux operators */
  orc_csr Mv, Mp;              /* energy operators (filtered, symmetrised) */
  uint8_t *keep_v, *keep_p;    /* drop masks over Ahat and Z entries */
  int64_t nnz_z;
  uint8_t *dir;                /* Dirichlet velocity nodes */
  /* coarsening */
  uint8_t *is_cp;              /* n_p */
  orc_csr S;                   /* S sets (fine C indices) */
  int32_t *sdist;
  int32_t *order;              /* C^(p) in selection order */
  int64_t n_cp, n_alg3;
  uint8_t *cbar;               /* n_p */
  int64_t n_mid;
  uint8_t *is_cv;              /* n_v */
  int64_t n_cv, n_extra_v;
  /* transfers (pattern + values) */
  orc_csr Pv, Pp;
  double *energy_v, *energy_p, *rho_v, *rho_p;  /* iters+1 */
  int its_v, its_p;
  /* coarse level */
  orc_csr Ac, Bc;
  double *xv_c;                /* n_cv*dim */
  int32_t *p2v_c;              /* n_cp */
  /* Petrov-Galerkin restriction (pg): R_v^T on Pv's pattern, its trace, and
   * the coarse gradient block's transpose on Bc's pattern */
  orc_csr Rvt, Gct;
  double *energy_r, *rho_r;    /* iters+1 */
  int its_r;
} orc_level_t;

/* options of orc_level_ex */
typedef struct {
  double tau1_v, tau1_p, tau2_sq;
  int iters;
  int energy_ata;              /* velocity P in the A^T A-norm */
  int gmres;                   /* velocity P by the GMRES form on A~ */
  int pg;                      /* Petrov-Galerkin restriction */
  const uint8_t *cp_in;        /* C^(p) given (n_p flags) or NULL */
} orc_opts_t;

/* Petrov-Galerkin Galerkin product: Ac = Rvt^T Ahat Pv, Bc = Pp^T Bdiv (I_d (x) Pv),
 * Gct = Pp^T Gt (I_d (x) Rvt) (Gt_val: values on Bdiv's pattern, NULL = Bdiv). */
int orc_rap_pg(const orc_csr *Ahat, const orc_csr *Bdiv, const double *Gt_val, int dim,
               const orc_csr *Pv, const orc_csr *Rvt, const orc_csr *Pp, orc_csr *Ac,
               orc_csr *Bc, orc_csr *Gct);

int orc_level(int dim, const orc_csr *Ahat, const orc_csr *Bdiv,
              const double *xv, const int32_t *p2v,
              double tau1_v, double tau1_p, double tau2_sq, int iters, int energy_ata,
              orc_level_t *out);
/* The same level with C^(p) given (cp_in, n_p flags) instead of chosen by
 * Alg. 3; NULL cp_in is orc_level. */
int orc_level_cp(int dim, const orc_csr *Ahat, const orc_csr *Bdiv,
                 const double *xv, const int32_t *p2v,
                 double tau1_v, double tau1_p, double tau2_sq, int iters, int energy_ata,
                 const uint8_t *cp_in, orc_level_t *L);
/* The level under options; Gt_val: the fine gradient block's transpose on
 * Bdiv's pattern (pg only; NULL = Bdiv). */
int orc_level_ex(int dim, const orc_csr *Ahat, const orc_csr *Bdiv, const double *Gt_val,
                 const double *xv, const int32_t *p2v, const orc_opts_t *o, orc_level_t *L);
void orc_level_free(orc_level_t *L);

#ifdef __cplusplus
}
#endif
#endif
