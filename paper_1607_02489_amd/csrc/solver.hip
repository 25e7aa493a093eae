// Solve phase on a hierarchy (sec. 5.2, sec. 6): Braess-Sarazin relaxation
// of eq. (bs), the multigrid V-cycle it smooths, and GMRES preconditioned on
// the right by that V-cycle.
//
// A level's operator is the saddle-point matrix
//   K = [ I_d (x) A   B^T ]
//       [ B           0   ]
// on vectors x = (u, p), u component-blocked.  One Braess-Sarazin step solves
// [D/omega, B^T; B, 0] delta = f - K x with D = diag(sum_j |a_ij|): the
// pressure part from the explicitly formed Schur complement S = B D^-1 B^T by
// forward Gauss-Seidel sweeps from zero, then
//   delta_u = (omega D^-1) (r_u - B^T delta_p).
// Gauss-Seidel keeps its sequential definition (each row takes the newest
// values of the rows before it): the rows are grouped by dependency level
// (a row's level is one more than the highest level among the earlier rows
// it couples to), rows of one level are updated together, levels in order,
// by one workgroup; a row sums its entries in ascending column order.  Every
// other sum has a fixed order too, so results are deterministic.
#include "common.h"

#include <cmath>
#include <vector>

namespace emin {
namespace {

constexpr int SB = 256;

__device__ __forceinline__ double blk_sum(double v, double* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) t += lds[k];
  return t;
}

// dinv_i = 1 / sum_j |a_ij| (0 for an empty row)
__global__ void k_bs_dinv(const int64_t* rp, const double* val, int64_t n, double* dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t e = rp[i]; e < rp[i + 1]; e++) s = s + fabs(val[e]);
  dinv[i] = s != 0.0 ? 1.0 / s : 0.0;
}

// rows r of B^T (velocity dofs, component-blocked) scaled by dinv[r mod nv]
__global__ void k_scale_rows_mod(const int64_t* rp, double* val, int64_t nrows, int64_t nv,
                                 const double* dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const double d = dinv[r % nv];
  for (int64_t e = rp[r]; e < rp[r + 1]; e++) val[e] = val[e] * d;
}

// position of each row's diagonal entry (-1 when absent)
__global__ void k_find_diag(const int64_t* rp, const int32_t* col, int64_t n, int64_t* pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t p = -1;
  for (int64_t e = rp[i]; e < rp[i + 1]; e++)
    if (col[e] == i) p = e;
  pos[i] = p;
}

// Gauss-Seidel dependency levels, rows in order (one thread): a row's level
// is one more than the highest level of the earlier rows in its pattern
__global__ void k_gs_levels(const int64_t* rp, const int32_t* col, int64_t n, int32_t* lev,
                            int32_t* nlev) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t top = 0;
  for (int64_t i = 0; i < n; i++) {
    int32_t l = 0;
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      const int32_t j = col[e];
      if (j >= i) break;   // (sorted columns)
      l = lev[j] + 1 > l ? lev[j] + 1 : l;
    }
    lev[i] = l;
    top = l + 1 > top ? l + 1 : top;
  }
  *nlev = top;
}

__global__ void k_level_count(const int32_t* lev, int64_t n, int64_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(reinterpret_cast<unsigned long long*>(cnt + lev[i] + 1), 1ull);
}

// rows placed by level (any order within a level: its rows are independent)
__global__ void k_level_place(const int32_t* lev, int64_t n, const int64_t* off, int32_t* cur,
                              int32_t* order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  order[off[lev[i]] + atomicAdd(&cur[lev[i]], 1)] = (int32_t)i;
}

// sweeps of forward Gauss-Seidel on S x = b, in place, one workgroup: the
// rows of a level together, levels in order (the workgroup's barrier orders
// a level's stores before the next level's loads); a row without a diagonal
// keeps its value
__global__ __launch_bounds__(1024) void k_gs(const int64_t* rp, const int32_t* col,
                                             const double* val, const int64_t* dpos,
                                             const int32_t* order, const int64_t* loff,
                                             int32_t nlev, const double* b, double* x,
                                             int sweeps) {
  for (int sw = 0; sw < sweeps; sw++)
    for (int32_t L = 0; L < nlev; L++) {
      for (int64_t t = loff[L] + threadIdx.x; t < loff[L + 1]; t += blockDim.x) {
        const int32_t i = order[t];
        const int64_t dp = dpos[i];
        double s = b[i];
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
          if (e != dp) s = s - val[e] * x[col[e]];
        const double di = dp >= 0 ? val[dp] : 0.0;
        x[i] = di != 0.0 ? s / di : 0.0;
      }
      __syncthreads();
    }
}

// velocity rows of r = f - K x (y = K x when f is null): row q = c nv + i
// sums A's row i over x_u's block c, then B^T's row q over x_p
__global__ void k_resid_u(const int64_t* arp, const int32_t* acol, const double* aval, int64_t nv,
                          int dim, const int64_t* btrp, const int32_t* btcol,
                          const double* btval, const double* x, const double* f, double* r) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= dim * nv) return;
  const int64_t c = q / nv, i = q - c * nv;
  const double* xu = x + c * nv;
  const double* xp = x + dim * nv;
  double s = 0.0;
  for (int64_t e = arp[i]; e < arp[i + 1]; e++) s = s + aval[e] * xu[acol[e]];
  double t = 0.0;
  for (int64_t e = btrp[q]; e < btrp[q + 1]; e++) t = t + btval[e] * xp[btcol[e]];
  s = s + t;
  r[q] = f ? f[q] - s : s;
}

// pressure rows of r = f - K x: B's row over x_u
__global__ void k_resid_p(const int64_t* brp, const int32_t* bcol, const double* bval, int64_t np,
                          int64_t nu, const double* x, const double* f, double* r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double s = 0.0;
  for (int64_t e = brp[i]; e < brp[i + 1]; e++) s = s + bval[e] * x[bcol[e]];
  r[nu + i] = f ? f[nu + i] - s : s;
}

// Braess-Sarazin right-hand side: rhs_i = sum_e b_e (dinv_c r_u,c) - r_p,i / omega
__global__ void k_bs_rhs(const int64_t* brp, const int32_t* bcol, const double* bval, int64_t np,
                         int64_t nv, int64_t nu, const double* dinv, const double* r,
                         double omega, double* rhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double s = 0.0;
  for (int64_t e = brp[i]; e < brp[i + 1]; e++) {
    const int32_t c = bcol[e];
    s = s + bval[e] * (dinv[c % nv] * r[c]);
  }
  rhs[i] = s - r[nu + i] / omega;
}

// x_u += (omega dinv) (r_u - B^T dp), x_p += dp
__global__ void k_bs_update(const int64_t* btrp, const int32_t* btcol, const double* btval,
                            int64_t nv, int64_t nu, int64_t np, const double* dinv, double omega,
                            const double* r, const double* dp, double* x) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nu) {
    double t = 0.0;
    for (int64_t e = btrp[q]; e < btrp[q + 1]; e++) t = t + btval[e] * dp[btcol[e]];
    x[q] = x[q] + (omega * dinv[q % nv]) * (r[q] - t);
  } else if (q < nu + np) {
    x[q] = x[q] + dp[q - nu];
  }
}

// y[b nrows + i] = (y +) sum_e m_e x[b ncols + col_e] for blocks b < nblk
__global__ void k_spmv_blocks(const int64_t* rp, const int32_t* col, const double* val,
                              int64_t nrows, int64_t ncols, int nblk, const double* x, double* y,
                              int add) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nrows * nblk) return;
  const int64_t b = q / nrows, i = q - b * nrows;
  const double* xb = x + b * ncols;
  double s = 0.0;
  for (int64_t e = rp[i]; e < rp[i + 1]; e++) s = s + val[e] * xb[col[e]];
  y[q] = add ? y[q] + s : s;
}

__global__ void k_fill(double* x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// partial sums of <a, b> per block of SB entries
__global__ __launch_bounds__(SB) void k_dot_part(const double* a, const double* b, int64_t n,
                                                 double* part) {
  __shared__ double lds[SB / 64];
  const int64_t e = (int64_t)blockIdx.x * SB + threadIdx.x;
  const double t = blk_sum(e < n ? a[e] * b[e] : 0.0, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// fixed-order sum of the partials into *out
__global__ __launch_bounds__(1024) void k_dot_fin(const double* part, int np, double* out) {
  __shared__ double lds[16];
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) v += part[k];
  const double t = blk_sum(v, lds);
  if (threadIdx.x == 0) *out = t;
}

// y = a / sqrt(*nrm2) (y = a when the norm is 0)
__global__ void k_scale_inv_norm(const double* a, const double* nrm2, int64_t n, double* y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double s = sqrt(*nrm2);
  y[e] = s > 0.0 ? a[e] / s : a[e];
}

// w -= h * v (h on the device)
__global__ void k_axpy_dev(double* w, const double* v, const double* h, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) w[e] = w[e] - (*h) * v[e];
}

// GMRES bookkeeping of column j (one thread): H[j+1][j] = sqrt(nrm2), the
// earlier rotations applied to column j, the new rotation, the residual
// estimate |g[j+1]| into *res
__global__ void k_gm_givens(double* H, int m, int j, const double* nrm2, double* cs, double* sn,
                            double* g, double* res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  H[(int64_t)(j + 1) * m + j] = sqrt(*nrm2);
  for (int i = 0; i < j; i++) {
    const double a = H[(int64_t)i * m + j], b = H[(int64_t)(i + 1) * m + j];
    H[(int64_t)i * m + j] = cs[i] * a + sn[i] * b;
    H[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[(int64_t)j * m + j], b = H[(int64_t)(j + 1) * m + j];
  const double r = sqrt(a * a + b * b);
  cs[j] = r > 0.0 ? a / r : 1.0;
  sn[j] = r > 0.0 ? b / r : 0.0;
  H[(int64_t)j * m + j] = r;
  H[(int64_t)(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  *res = fabs(g[j + 1]);
}

// back substitution of the k x k upper triangle (one thread)
__global__ void k_gm_backsub(const double* H, int m, int k, const double* g, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; i--) {
    double t = g[i];
    for (int c = i + 1; c < k; c++) t = t - H[(int64_t)i * m + c] * y[c];
    y[i] = t / H[(int64_t)i * m + i];
  }
}

// z = sum_i y_i v_i (ascending i)
__global__ void k_combine(const double* V, int64_t n, const double* y, int k, double* z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; i++) s = s + y[i] * V[(int64_t)i * n + e];
  z[e] = s;
}

__global__ void k_set_g0(const double* nrm2, double* g) {
  if (threadIdx.x == 0 && blockIdx.x == 0) g[0] = sqrt(*nrm2);
}

}  // namespace
}  // namespace emin

using namespace emin;

struct SolverLevel {
  int dim = 2;
  int64_t nv = 0, np = 0, nu = 0, n = 0;
  CsrView A, B;            // borrowed (level 0: the caller's; coarse: the hierarchy's)
  Csr BT;                  // B^T with values
  double* dinv = nullptr;  // nv
  Csr S;                   // B D^-1 B^T
  int64_t* dpos = nullptr;
  int32_t* order = nullptr;
  int64_t* loff = nullptr;
  int32_t nlev = 0;
  // transfer to the next coarser level (absent on the coarsest)
  bool has_p = false;
  CsrView P, Pp;           // n_v x n_vc, n_p x n_pc
  Csr PT, PpT;
  int64_t nvc = 0, npc = 0;
  double *x = nullptr, *f = nullptr, *r = nullptr, *rhs = nullptr, *dp = nullptr;
};

struct emin_solver_s {
  Arena ar;
  std::vector<SolverLevel> L;
  int32_t nu = 2, sweeps = 5, coarse_steps = 10;
  double omega = 0.666;
  double* part = nullptr;
  int64_t npart = 0;
  double* scal = nullptr;   // device scalars
  // GMRES workspace (grown on demand)
  int32_t gm_cap = 0;
  double *V = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr,
         *w = nullptr, *z = nullptr;
};

namespace {

unsigned nb(int64_t n) { return nblocks(n > 0 ? n : 1, SB); }

Csr transpose_with_values(const CsrView& M, hipStream_t s, Arena& ar) {
  Csr T;
  int32_t* src = nullptr;
  transpose_pattern(M, T, src, s, ar);
  T.val = ar.alloc<double>(T.nnz);
  if (T.nnz) gather_values(M.val, src, T.val, T.nnz, s);
  return T;
}

void dot(emin_solver_t* S, const double* a, const double* b, int64_t n, double* out,
         hipStream_t s) {
  const unsigned np = nb(n);
  k_dot_part<<<np, SB, 0, s>>>(a, b, n, S->part);
  k_dot_fin<<<1, 1024, 0, s>>>(S->part, (int)np, out);
}

void residual(const SolverLevel& L, const double* x, const double* f, double* r, hipStream_t s) {
  k_resid_u<<<nb(L.nu), SB, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, L.nv, L.dim, L.BT.rowptr,
                                     L.BT.col, L.BT.val, x, f, r);
  k_resid_p<<<nb(L.np), SB, 0, s>>>(L.B.rowptr, L.B.col, L.B.val, L.np, L.nu, x, f, r);
}

void bs_step(emin_solver_t* S, SolverLevel& L, double* x, const double* f, hipStream_t s) {
  residual(L, x, f, L.r, s);
  k_bs_rhs<<<nb(L.np), SB, 0, s>>>(L.B.rowptr, L.B.col, L.B.val, L.np, L.nv, L.nu, L.dinv, L.r,
                                    S->omega, L.rhs);
  k_fill<<<nb(L.np), SB, 0, s>>>(L.dp, L.np, 0.0);
  if (L.np && L.nlev)
    k_gs<<<1, 1024, 0, s>>>(L.S.rowptr, L.S.col, L.S.val, L.dpos, L.order, L.loff, L.nlev,
                            L.rhs, L.dp, S->sweeps);
  k_bs_update<<<nb(L.n), SB, 0, s>>>(L.BT.rowptr, L.BT.col, L.BT.val, L.nv, L.nu, L.np, L.dinv,
                                      S->omega, L.r, L.dp, x);
}

// x = V-cycle(f) on level l, from x = 0 (x, f: level-l vectors)
void vcycle(emin_solver_t* S, int l, const double* f, double* x, hipStream_t s) {
  SolverLevel& L = S->L[l];
  k_fill<<<nb(L.n), SB, 0, s>>>(x, L.n, 0.0);
  if (l + 1 == (int)S->L.size()) {
    for (int k = 0; k < S->coarse_steps; k++) bs_step(S, L, x, f, s);
    return;
  }
  for (int k = 0; k < S->nu; k++) bs_step(S, L, x, f, s);
  SolverLevel& C = S->L[l + 1];
  residual(L, x, f, L.r, s);
  // f_c = (P^T r_u per component, Pp^T r_p)
  k_spmv_blocks<<<nb(L.dim * L.nvc), SB, 0, s>>>(L.PT.rowptr, L.PT.col, L.PT.val, L.nvc, L.nv,
                                                  L.dim, L.r, C.f, 0);
  k_spmv_blocks<<<nb(L.npc), SB, 0, s>>>(L.PpT.rowptr, L.PpT.col, L.PpT.val, L.npc, L.np, 1,
                                          L.r + L.nu, C.f + C.nu, 0);
  vcycle(S, l + 1, C.f, C.x, s);
  // x += (P x_c,u per component, Pp x_c,p)
  k_spmv_blocks<<<nb(L.nu), SB, 0, s>>>(L.P.rowptr, L.P.col, L.P.val, L.nv, L.nvc, L.dim, C.x,
                                         x, 1);
  k_spmv_blocks<<<nb(L.np), SB, 0, s>>>(L.Pp.rowptr, L.Pp.col, L.Pp.val, L.np, L.npc, 1,
                                         C.x + C.nu, x + L.nu, 1);
  for (int k = 0; k < S->nu; k++) bs_step(S, L, x, f, s);
}

void setup_level(emin_solver_t* S, SolverLevel& L, hipStream_t s) {
  Arena& ar = S->ar;
  L.nu = L.dim * L.nv;
  L.n = L.nu + L.np;
  L.BT = transpose_with_values(L.B, s, ar);
  L.dinv = ar.alloc<double>(L.nv);
  if (L.nv) k_bs_dinv<<<nb(L.nv), SB, 0, s>>>(L.A.rowptr, L.A.val, L.nv, L.dinv);
  // S = B (D^-1 B^T)
  Csr DBT = L.BT;
  DBT.val = ar.alloc<double>(L.BT.nnz);
  if (L.BT.nnz) {
    HIP_OK(hipMemcpyAsync(DBT.val, L.BT.val, sizeof(double) * L.BT.nnz, hipMemcpyDeviceToDevice,
                          s));
    k_scale_rows_mod<<<nb(L.nu), SB, 0, s>>>(DBT.rowptr, DBT.val, L.nu, L.nv, L.dinv);
  }
  SpgemmPlan plan;
  spgemm_symbolic(L.B, view(DBT), L.S, plan, s, ar, nullptr);
  L.S.val = ar.alloc<double>(L.S.nnz);
  spgemm_numeric(L.B, view(DBT), L.S, plan, s);
  // Gauss-Seidel levels
  L.dpos = ar.alloc<int64_t>(L.np);
  int32_t* lev = ar.alloc<int32_t>(L.np);
  int32_t* dn = ar.alloc<int32_t>(1);
  HIP_OK(hipMemsetAsync(dn, 0, sizeof(int32_t), s));
  if (L.np) {
    k_find_diag<<<nb(L.np), SB, 0, s>>>(L.S.rowptr, L.S.col, L.np, L.dpos);
    k_gs_levels<<<1, 64, 0, s>>>(L.S.rowptr, L.S.col, L.np, lev, dn);
  }
  L.nlev = d2h(dn, s);
  L.loff = ar.alloc<int64_t>((size_t)L.nlev + 1);
  HIP_OK(hipMemsetAsync(L.loff, 0, sizeof(int64_t) * ((size_t)L.nlev + 1), s));
  L.order = ar.alloc<int32_t>(L.np);
  int32_t* cur = ar.alloc<int32_t>(L.nlev > 0 ? L.nlev : 1);
  HIP_OK(hipMemsetAsync(cur, 0, sizeof(int32_t) * (L.nlev > 0 ? L.nlev : 1), s));
  if (L.np && L.nlev) {
    k_level_count<<<nb(L.np), SB, 0, s>>>(lev, L.np, L.loff);
    scan_inclusive(L.loff + 1, L.nlev, s, ar);
    k_level_place<<<nb(L.np), SB, 0, s>>>(lev, L.np, L.loff, cur, L.order);
  }
  if (L.has_p) {
    L.PT = transpose_with_values(L.P, s, ar);
    L.PpT = transpose_with_values(L.Pp, s, ar);
  }
  L.x = ar.alloc<double>(L.n);
  L.f = ar.alloc<double>(L.n);
  L.r = ar.alloc<double>(L.n);
  L.rhs = ar.alloc<double>(L.np);
  L.dp = ar.alloc<double>(L.np);
}

template <class F>
emin_status guard(F&& f) {
  try {
    f();
    return EMIN_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (...) {
    return EMIN_ERR_DEVICE;
  }
}

CsrView view_of(const emin_view_t& v, const double* val) {
  return {v.n, v.ncols, v.nnz, v.rowptr, v.col, val};
}

}  // namespace

extern "C" {

emin_status emin_solver_create(const emin_system_t* sys, const emin_hierarchy_t* h, int32_t nu,
                               double omega, int32_t gs_sweeps, int32_t coarse_steps,
                               void* stream, emin_solver_t** out) {
  if (!out) return EMIN_ERR_ARG;
  *out = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  emin_solver_t* S = nullptr;
  const emin_status st = guard([&] {
    if (!sys || !h || nu < 0 || gs_sweeps < 0 || coarse_steps < 0 || !(omega > 0.0))
      throw Error(EMIN_ERR_ARG, "parameter");
    int32_t nt = 0;
    if (emin_hierarchy_info(h, &nt, nullptr, 0) != EMIN_OK) throw Error(EMIN_ERR_ARG, "hierarchy");
    S = new emin_solver_s();
    S->nu = nu;
    S->omega = omega;
    S->sweeps = gs_sweeps;
    S->coarse_steps = coarse_steps;
    S->L.resize((size_t)nt + 1);
    const int dim = sys->dim;
    CsrView A{sys->Ahat.nrows, sys->Ahat.ncols, sys->Ahat.nnz, sys->Ahat.rowptr, sys->Ahat.col,
              sys->Ahat.val};
    CsrView B{sys->Bdiv.nrows, sys->Bdiv.ncols, sys->Bdiv.nnz, sys->Bdiv.rowptr, sys->Bdiv.col,
              sys->Bdiv.val};
    for (int32_t l = 0; l <= nt; l++) {
      SolverLevel& L = S->L[l];
      L.dim = dim;
      L.A = A;
      L.B = B;
      L.nv = A.nrows;
      L.np = B.nrows;
      if (B.ncols != dim * L.nv || A.ncols != L.nv)
        throw Error(EMIN_ERR_SHAPE, "level operators do not match");
      if (l == nt) break;
      emin_pattern_t* pat = nullptr;
      const double *Pv, *Pp, *Ac, *Bc;
      if (emin_hierarchy_level(h, l, &pat, &Pv, &Pp, &Ac, &Bc, nullptr) != EMIN_OK)
        throw Error(EMIN_ERR_ARG, "hierarchy level");
      emin_view_t vp, vpp, vac, vbc;
      if (emin_pattern_view(pat, EMIN_VIEW_PV, &vp) != EMIN_OK ||
          emin_pattern_view(pat, EMIN_VIEW_PP, &vpp) != EMIN_OK ||
          emin_pattern_view(pat, EMIN_VIEW_AC, &vac) != EMIN_OK ||
          emin_pattern_view(pat, EMIN_VIEW_BC, &vbc) != EMIN_OK)
        throw Error(EMIN_ERR_ARG, "pattern views");
      L.has_p = true;
      L.P = view_of(vp, Pv);
      L.Pp = view_of(vpp, Pp);
      L.nvc = vp.ncols;
      L.npc = vpp.ncols;
      A = view_of(vac, Ac);
      B = view_of(vbc, Bc);
    }
    for (int32_t l = 0; l < nt; l++)
      if (S->L[l].nvc != S->L[l + 1].nv || S->L[l].npc != S->L[l + 1].np)
        throw Error(EMIN_ERR_SHAPE, "transfer does not match the coarse level");
    int64_t nmax = 1;
    for (SolverLevel& L : S->L) {
      setup_level(S, L, s);
      nmax = L.n > nmax ? L.n : nmax;
    }
    S->npart = nb(nmax);
    S->part = S->ar.alloc<double>(S->npart);
    S->scal = S->ar.alloc<double>(8);
    HIP_OK(hipStreamSynchronize(s));
  });
  if (st != EMIN_OK) {
    (void)hipStreamSynchronize(s);
    delete S;
    return st;
  }
  *out = S;
  return EMIN_OK;
}

emin_status emin_solver_info(const emin_solver_t* S, int32_t level, int64_t* n, int32_t* gs_levels) {
  if (!S || level < 0 || level >= (int32_t)S->L.size()) return EMIN_ERR_ARG;
  if (n) *n = S->L[level].n;
  if (gs_levels) *gs_levels = S->L[level].nlev;
  return EMIN_OK;
}

emin_status emin_solver_bs_step(emin_solver_t* S, int32_t level, double* x, const double* f,
                                void* stream) {
  if (!S || level < 0 || level >= (int32_t)S->L.size() || !x || !f) return EMIN_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    bs_step(S, S->L[level], x, f, s);
    HIP_OK(hipGetLastError());
  });
}

emin_status emin_solver_vcycle(emin_solver_t* S, const double* f, double* x, void* stream) {
  if (!S || !f || !x) return EMIN_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    StreamUse use_ar(S->ar, s);
    vcycle(S, 0, f, x, s);
    HIP_OK(hipGetLastError());
  });
}

emin_status emin_solver_gmres(emin_solver_t* S, const double* f, double* x, double rtol,
                              int32_t maxit, int32_t* its, double* relres, void* stream) {
  if (!S || !f || !x || maxit < 1 || !(rtol >= 0.0)) return EMIN_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    StreamUse use_ar(S->ar, s);
    const SolverLevel& L0 = S->L[0];
    const int64_t n = L0.n;
    const int m = maxit;
    if (m > S->gm_cap) {
      S->V = S->ar.alloc<double>((size_t)(m + 1) * (size_t)(n > 0 ? n : 1));
      S->H = S->ar.alloc<double>((size_t)(m + 1) * m);
      S->cs = S->ar.alloc<double>(m);
      S->sn = S->ar.alloc<double>(m);
      S->g = S->ar.alloc<double>(m + 1);
      S->y = S->ar.alloc<double>(m);
      S->w = S->ar.alloc<double>(n);
      S->z = S->ar.alloc<double>(n);
      S->gm_cap = m;
    }
    double* nrm2 = S->scal;
    double* res = S->scal + 1;
    HIP_OK(hipMemsetAsync(S->H, 0, sizeof(double) * (size_t)(m + 1) * m, s));
    HIP_OK(hipMemsetAsync(S->g, 0, sizeof(double) * (m + 1), s));
    dot(S, f, f, n, nrm2, s);
    k_set_g0<<<1, 64, 0, s>>>(nrm2, S->g);
    k_scale_inv_norm<<<nb(n), SB, 0, s>>>(f, nrm2, n, S->V);
    double beta2 = 0.0;
    HIP_OK(hipMemcpyAsync(&beta2, nrm2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double beta = std::sqrt(beta2);
    int k = 0;
    double last = beta;
    if (beta > 0.0) {
      for (int j = 0; j < m; j++) {
        const double* vj = S->V + (int64_t)j * n;
        vcycle(S, 0, vj, S->z, s);
        residual(L0, S->z, nullptr, S->w, s);   // w = K M v_j
        for (int i = 0; i <= j; i++) {
          const double* vi = S->V + (int64_t)i * n;
          double* hij = S->H + (int64_t)i * m + j;
          dot(S, vi, S->w, n, hij, s);
          k_axpy_dev<<<nb(n), SB, 0, s>>>(S->w, vi, hij, n);
        }
        dot(S, S->w, S->w, n, nrm2, s);
        k_gm_givens<<<1, 64, 0, s>>>(S->H, m, j, nrm2, S->cs, S->sn, S->g, res);
        k_scale_inv_norm<<<nb(n), SB, 0, s>>>(S->w, nrm2, n, S->V + (int64_t)(j + 1) * n);
        double rr[2];
        HIP_OK(hipMemcpyAsync(rr, S->scal, sizeof(rr), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        k = j + 1;
        last = rr[1];
        if (rr[1] <= rtol * beta || !(rr[0] > 0.0)) break;
      }
      k_gm_backsub<<<1, 64, 0, s>>>(S->H, m, k, S->g, S->y);
      k_combine<<<nb(n), SB, 0, s>>>(S->V, n, S->y, k, S->w);
      vcycle(S, 0, S->w, x, s);
    } else {
      k_fill<<<nb(n), SB, 0, s>>>(x, n, 0.0);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    if (its) *its = k;
    if (relres) *relres = beta > 0.0 ? last / beta : 0.0;
  });
}

void emin_solver_destroy(emin_solver_t* S) { delete S; }

}  // extern "C"
