// The GMRES form of the constrained minimisation (sec. 4.3, eq. (min_problem)
// for a non-symmetric operator): k steps of GMRES on the projected masked
// system Pi mask_N(K P) = 0 from the same feasible start P0 as the CG form.
// The iterate minimises ||Pi mask_N(K P)||_F over P0 + K_k(Pi mask_N(K .), R0).
//
// Device layout: the Krylov basis V (k+1 vectors over P's pattern entries),
// the Hessenberg matrix H ((k+1) x k, row-major), the state (beta, steps
// taken, stop flag).  Every inner product is a fixed two-level tree (block
// partials, then one block), so results do not depend on scheduling.  The
// small least-squares problem (Givens rotations, back substitution) runs in
// one thread at the end.
#include "emin_cg.h"

namespace emin {

namespace {

constexpr int GB = 256;   // block size of the vector kernels

struct GmState {
  double beta;
  int32_t its;    // Arnoldi steps completed
  int32_t stop;   // the residual vanished (no further steps)
};

__device__ __forceinline__ double gm_block_sum(double v, double* lds) {
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

// partial sums of <a, b>, one per block of GB entries
__global__ __launch_bounds__(GB) void k_gm_dot(const double* a, const double* b, int64_t n,
                                               double* part) {
  __shared__ double lds[GB / 64];
  const int64_t e = (int64_t)blockIdx.x * GB + threadIdx.x;
  const double v = e < n ? a[e] * b[e] : 0.0;
  const double t = gm_block_sum(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// fixed-order sum of the partials; what to do with it by mode
enum { GM_BETA = 0, GM_H = 1, GM_NORM = 2 };
__global__ __launch_bounds__(1024) void k_gm_fin(const double* part, int np, int mode, int i,
                                                 int j, int m, double* H, GmState* st,
                                                 double* rep_rho) {
  __shared__ double lds[16];
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) v += part[k];
  const double tot = gm_block_sum(v, lds);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case GM_BETA:
      st->beta = sqrt(tot);
      st->its = 0;
      st->stop = tot > 0.0 ? 0 : 1;
      if (rep_rho) rep_rho[0] = tot;
      break;
    case GM_H:
      H[(int64_t)i * m + j] = st->stop ? 0.0 : tot;
      break;
    case GM_NORM:
      if (!st->stop) {
        const double hn = sqrt(tot);
        H[(int64_t)(j + 1) * m + j] = hn;
        st->its = j + 1;
        if (!(hn > 0.0)) st->stop = 1;
      }
      break;
  }
}

// Pi on every row of X (in place): C rows to 0, an F row loses its component
// along W_c restricted to the row
__global__ __launch_bounds__(GB) void k_gm_project(const int64_t* rp, const int32_t* col,
                                                   int64_t n, const int32_t* cid,
                                                   const double* Wc, const double* G, double* X) {
  const int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x;
  if (i >= n) return;
  const int64_t a = rp[i], b = rp[i + 1];
  if (cid[i] >= 0) {
    for (int64_t s = a; s < b; s++) X[s] = 0.0;
    return;
  }
  if (!(G[i] > 0.0)) return;
  double dot = 0.0;
  for (int64_t s = a; s < b; s++) dot = dot + X[s] * Wc[col[s]];
  const double f = dot / G[i];
  for (int64_t s = a; s < b; s++) X[s] = X[s] - f * Wc[col[s]];
}

__global__ __launch_bounds__(GB) void k_gm_neg(double* X, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * GB + threadIdx.x;
  if (e < n) X[e] = -X[e];
}

// dst = src / d, d = beta (j < 0) or H[j+1][j]; skipped once stopped
__global__ __launch_bounds__(GB) void k_gm_scale(double* dst, const double* src, int64_t n,
                                                 const double* H, int j, int m,
                                                 const GmState* st) {
  const int64_t e = (int64_t)blockIdx.x * GB + threadIdx.x;
  if (e >= n || st->stop) return;
  const double d = j < 0 ? st->beta : H[(int64_t)(j + 1) * m + j];
  dst[e] = src[e] / d;
}

// X -= H[i][j] * v_i
__global__ __launch_bounds__(GB) void k_gm_axpy(double* X, const double* vi, int64_t n,
                                                const double* H, int i, int j, int m) {
  const int64_t e = (int64_t)blockIdx.x * GB + threadIdx.x;
  if (e >= n) return;
  X[e] = X[e] - H[(int64_t)i * m + j] * vi[e];
}

// Givens rotations over the completed columns, residual norms (squared) per
// step into the report, back substitution y; one thread
__global__ void k_gm_solve(double* H, int m, const GmState* st, double* y, double* rep_rho,
                           int32_t* rep_its) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = st->its;
  double cs[EMIN_MAX_ITERS], sn[EMIN_MAX_ITERS], g[EMIN_MAX_ITERS + 1];
  for (int t = 0; t <= m; t++) g[t] = 0.0;
  g[0] = st->beta;
  for (int j = 0; j < k; j++) {
    for (int i = 0; i < j; i++) {
      const double a = H[(int64_t)i * m + j], b = H[(int64_t)(i + 1) * m + j];
      H[(int64_t)i * m + j] = cs[i] * a + sn[i] * b;
      H[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
    }
    const double a = H[(int64_t)j * m + j], b = H[(int64_t)(j + 1) * m + j];
    const double r = sqrt(a * a + b * b);
    cs[j] = a / r;
    sn[j] = b / r;
    H[(int64_t)j * m + j] = r;
    H[(int64_t)(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    if (rep_rho) rep_rho[j + 1] = g[j + 1] * g[j + 1];
  }
  for (int i = k - 1; i >= 0; i--) {
    double t = g[i];
    for (int c = i + 1; c < k; c++) t = t - H[(int64_t)i * m + c] * y[c];
    y[i] = t / H[(int64_t)i * m + i];
  }
  if (rep_its) *rep_its = k;
}

// P += sum over the completed steps of y_i v_i (in step order)
__global__ __launch_bounds__(GB) void k_gm_update(double* P, const double* V, int64_t n,
                                                  const double* y, const GmState* st) {
  const int64_t e = (int64_t)blockIdx.x * GB + threadIdx.x;
  if (e >= n) return;
  double p = P[e];
  for (int i = 0; i < st->its; i++) p = p + y[i] * V[(int64_t)i * n + e];
  P[e] = p;
}

}  // namespace

void run_emin_gmres(EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp,
                    const int32_t* ncol, const int32_t* cid, const int32_t* clist, const double* W,
                    double* P, int iters, bool mixed, EminReportPtrs rp, GmresWork& gw,
                    hipStream_t s) {
  const int64_t n = w.n, nnz = w.nnz;
  if (n == 0) return;
  if (iters > gw.cap) throw Error(EMIN_ERR_ARG, "GMRES workspace smaller than iters");
  const int m = iters > 0 ? iters : 1;
  GmState* st = reinterpret_cast<GmState*>(gw.state);
  double* V = gw.V;
  double* H = gw.H;
  double* part = w.part;
  const unsigned nbv = nblocks(nnz, GB);
  const unsigned nbr = nblocks(n, GB);
  if (w.nc && clist) gather_modes(W, clist, w.nc, w.Wc, s);
  emin_init(nrp, ncol, n, nnz, cid, W, w.Wc, w.G, P, rp.status, s);
  // R0 = -Pi mask(K P0) into v_0, beta = ||R0||
  masked_product(w, M, Mf, nrp, ncol, P, V, mixed, s);
  if (nnz) {
    k_gm_neg<<<nbv, GB, 0, s>>>(V, nnz);
    k_gm_project<<<nbr, GB, 0, s>>>(nrp, ncol, n, cid, w.Wc, w.G, V);
    k_gm_dot<<<nbv, GB, 0, s>>>(V, V, nnz, part);
  }
  k_gm_fin<<<1, 1024, 0, s>>>(part, (int)nbv, GM_BETA, 0, 0, m, H, st, rp.rho);
  if (nnz) k_gm_scale<<<nbv, GB, 0, s>>>(V, V, nnz, H, -1, m, st);
  double* Qv = w.Q;
  for (int j = 0; j < iters; j++) {
    const double* vj = V + (int64_t)j * nnz;
    masked_product(w, M, Mf, nrp, ncol, vj, Qv, mixed, s);
    if (nnz) k_gm_project<<<nbr, GB, 0, s>>>(nrp, ncol, n, cid, w.Wc, w.G, Qv);
    for (int i = 0; i <= j; i++) {
      const double* vi = V + (int64_t)i * nnz;
      if (nnz) k_gm_dot<<<nbv, GB, 0, s>>>(vi, Qv, nnz, part);
      k_gm_fin<<<1, 1024, 0, s>>>(part, (int)nbv, GM_H, i, j, m, H, st, nullptr);
      if (nnz) k_gm_axpy<<<nbv, GB, 0, s>>>(Qv, vi, nnz, H, i, j, m);
    }
    if (nnz) k_gm_dot<<<nbv, GB, 0, s>>>(Qv, Qv, nnz, part);
    k_gm_fin<<<1, 1024, 0, s>>>(part, (int)nbv, GM_NORM, 0, j, m, H, st, nullptr);
    if (nnz) k_gm_scale<<<nbv, GB, 0, s>>>(V + (int64_t)(j + 1) * nnz, Qv, nnz, H, j, m, st);
  }
  k_gm_solve<<<1, 64, 0, s>>>(H, m, st, gw.y, rp.rho, rp.its);
  if (nnz) k_gm_update<<<nbv, GB, 0, s>>>(P, V, nnz, gw.y, st);
}

void GmresWork::reserve(int iters, int64_t nnz, int64_t np, Arena& ar) {
  if (iters <= cap && V) return;
  cap = iters;
  V = ar.alloc<double>((size_t)(iters + 1) * (size_t)(nnz > 0 ? nnz : 1));
  H = ar.alloc<double>((size_t)(iters + 1) * (size_t)(iters > 0 ? iters : 1));
  y = ar.alloc<double>(iters > 0 ? iters : 1);
  state = ar.alloc<double>(2);
  (void)np;
}

}  // namespace emin
