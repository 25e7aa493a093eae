// Inf-sup diagnostic of sec. 6.1 (Table 3): the smallest non-zero singular
// value of the mass-scaled divergence
//   B~ = lump(|M_p|)^(-1/2) B lump(|M_v|)^(-1/2)
// on each level, with the mass matrices projected down the hierarchy by the
// level's own transfers (M_{l+1} = R M_l P).
//
// sigma_min^2 is the smallest non-zero eigenvalue of S = B~ B~^T (n_p x n_p).
// S is applied as two sparse products (with B^T and with B) and a diagonal
// scaling, never formed.  Lanczos with full re-orthogonalisation (classical
// Gram-Schmidt, twice) builds the tridiagonal T_m; its eigenvalues are found
// by Sturm-count bisection in one thread, and those below rel * lambda_max
// count as zero (the hydrostatic pressure of an enclosed flow).  With
// m = n_p - 1 steps the Ritz values are S's eigenvalues; with fewer, the
// smallest non-zero one converges from above.  Every inner product is a
// fixed tree, so the result does not depend on scheduling.
#include "common.h"

#include <cmath>

struct emin_matrix_s {
  emin::Arena ar;
  emin::Csr C;
};

namespace emin {
namespace {

constexpr int IB = 256;

__device__ __forceinline__ double isum(double v, double* lds) {
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

// d_i = sum_j |m_ij| (one row per thread)
__global__ void k_lump_abs(const int64_t* rp, const double* val, int64_t n, double* d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t e = rp[i]; e < rp[i + 1]; e++) s = s + fabs(val[e]);
  d[i] = s;
}

// y = D^{-1/2} x or y = D^{-1} x (pw = 1 or 2), D repeated every nd entries
__global__ void k_dscale(const double* x, const double* d, int64_t n, int64_t nd, int pw,
                         double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = d[i % nd];
  y[i] = pw == 2 ? x[i] / di : x[i] / sqrt(di);
}

// y = A x, one row per thread
__global__ void k_spmv(const int64_t* rp, const int32_t* col, const double* val, int64_t n,
                       const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t e = rp[i]; e < rp[i + 1]; e++) s = s + val[e] * x[col[e]];
  y[i] = s;
}

// c[i] = <q_i, w> for i < k: one block per basis vector, each thread a
// strided slice in ascending order, then the block's fixed tree
__global__ __launch_bounds__(IB) void k_qt_dot(const double* Q, const double* w, int64_t n,
                                               double* c) {
  __shared__ double lds[IB / 64];
  const double* q = Q + (int64_t)blockIdx.x * n;
  double v = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += IB) v = v + q[e] * w[e];
  const double t = isum(v, lds);
  if (threadIdx.x == 0) c[blockIdx.x] = t;
}

// w -= sum_{i<k} c[i] q_i (ascending i)
__global__ void k_multi_axpy(const double* Q, int k, const double* c, int64_t n, double* w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double x = w[e];
  for (int i = 0; i < k; i++) x = x - c[i] * Q[(int64_t)i * n + e];
  w[e] = x;
}

// Lanczos bookkeeping of step j: alpha_j = <q_j, S q_j> (c[j] of the first
// projection), beta_j = ||w|| after re-orthogonalisation; q_{j+1} = w / beta_j
__global__ void k_lz_scalars(const double* c, int j, const double* nrm2, double* alpha,
                             double* beta, int* stop) {
  // stop[0]: the Krylov space became invariant; stop[1]: steps in T
  if (threadIdx.x != 0 || stop[0]) return;
  alpha[j] = c[j];
  const double b = sqrt(*nrm2);
  beta[j] = b;
  stop[1] = j + 1;
  if (!(b > 0.0)) stop[0] = 1;
}

__global__ void k_lz_next(const double* w, const double* beta, int j, const int* stop, int64_t n,
                          double* qn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n || *stop) return;
  qn[e] = w[e] / beta[j];
}

// deterministic start vector: 1 + (a hash of i) / 2^32, normalised later
__global__ void k_lz_start(int64_t n, double* q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t x = (uint32_t)i * 2654435761u + 12345u;
  x ^= x >> 15;
  x *= 2246822519u;
  x ^= x >> 13;
  q[i] = 1.0 + (double)x * (1.0 / 4294967296.0);
}

__global__ void k_scale_by(double* q, int64_t n, const double* nrm2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = q[i] / sqrt(*nrm2);
}

// Sturm count: eigenvalues of the tridiagonal (alpha, beta) below x
__device__ int sturm_below(const double* a, const double* b, int m, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < m; i++) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) cnt++;
  }
  return cnt;
}

// Solves (T - mu I) x = x in place for the tridiagonal T (diagonal a,
// off-diagonal b, order m) by Gaussian elimination with partial pivoting;
// wk holds 4 m doubles.  A zero pivot is replaced by a tiny one, as inverse
// iteration at an eigenvalue needs.
__device__ void tri_shift_solve(const double* a, const double* b, int m, double mu, double* x,
                                double* wk) {
  double *d = wk, *du = wk + m, *du2 = wk + 2 * m, *dl = wk + 3 * m;
  for (int i = 0; i < m; i++) {
    d[i] = a[i] - mu;
    du[i] = i + 1 < m ? b[i] : 0.0;
    dl[i] = i + 1 < m ? b[i] : 0.0;
    du2[i] = 0.0;
  }
  // elimination and forward substitution of x in one sweep
  for (int i = 0; i + 1 < m; i++) {
    if (fabs(d[i]) >= fabs(dl[i])) {
      if (d[i] == 0.0) d[i] = 1e-300;
      const double f = dl[i] / d[i];
      dl[i] = f;
      d[i + 1] = d[i + 1] - f * du[i];
      // forward substitution of the right-hand side, no swap
      x[i + 1] = x[i + 1] - f * x[i];
    } else {
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = d[i + 1];
      d[i + 1] = t - f * d[i + 1];
      if (i + 2 < m) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
      const double xi = x[i];
      x[i] = x[i + 1];
      x[i + 1] = xi - f * x[i];
    }
  }
  if (d[m - 1] == 0.0) d[m - 1] = 1e-300;
  for (int i = m - 1; i >= 0; i--) {
    double t = x[i];
    if (i + 1 < m) t = t - du[i] * x[i + 1];
    if (i + 2 < m) t = t - du2[i] * x[i + 2];
    x[i] = t / d[i];
  }
}

// Ritz values by bisection: lambda_max, the number below rel * lambda_max,
// the smallest one above it (theta), and the Lanczos residual of theta's
// Ritz vector, beta_m |s_m| with s theta's unit eigenvector of T (three
// steps of inverse iteration): an eigenvalue of the operator lies within
// that distance of theta.  One thread; wk holds 5 m doubles.
__global__ void k_lz_ritz(const double* a, const double* b, const int* mptr, double rel,
                          double* wk, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int m = *mptr;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; i++) {
    const double r = (i ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  auto kth = [&](int k) {   // k-th smallest (0-based)
    double l = lo, h = hi;
    for (int it = 0; it < 200; it++) {
      const double mid = 0.5 * (l + h);
      if (mid <= l || mid >= h) break;
      if (sturm_below(a, b, m, mid) > k) h = mid; else l = mid;
    }
    return 0.5 * (l + h);
  };
  const double lmax = m ? kth(m - 1) : 0.0;
  const int nzero = m ? sturm_below(a, b, m, rel * lmax) : 0;
  const double theta = nzero < m ? kth(nzero) : 0.0;
  out[0] = lmax;
  out[1] = (double)nzero;
  out[2] = theta;
  out[3] = 0.0;
  if (nzero >= m) return;
  double* x = wk + 4 * m;
  for (int i = 0; i < m; i++) x[i] = 1.0;
  for (int it = 0; it < 3; it++) {
    tri_shift_solve(a, b, m, theta, x, wk);
    double mx = 0.0;
    for (int i = 0; i < m; i++) mx = fmax(mx, fabs(x[i]));
    if (!(mx > 0.0) || !(mx < 1e300)) return;   // (out[3] stays 0: no estimate)
    double nn = 0.0;
    for (int i = 0; i < m; i++) {
      x[i] = x[i] / mx;
      nn = nn + x[i] * x[i];
    }
    const double inv = 1.0 / sqrt(nn);
    for (int i = 0; i < m; i++) x[i] = x[i] * inv;
  }
  out[3] = fabs(b[m - 1]) * fabs(x[m - 1]);
}

}  // namespace
}  // namespace emin

using namespace emin;

namespace {

CsrView viewof(const emin_csr_t& c) { return {c.nrows, c.ncols, c.nnz, c.rowptr, c.col, c.val}; }

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

void check_csr_arg(const emin_csr_t* a) {
  if (!a) throw Error(EMIN_ERR_ARG, "NULL matrix");
  if (a->nrows < 0 || a->ncols < 0 || a->nnz < 0) throw Error(EMIN_ERR_ARG, "negative size");
  if ((a->nrows && !a->rowptr) || (a->nnz && (!a->col || !a->val)))
    throw Error(EMIN_ERR_ARG, "NULL array");
}

}  // namespace

extern "C" {

emin_status emin_galerkin(const emin_csr_t* M, const emin_csr_t* P, void* stream,
                          emin_matrix_t** out) {
  if (!out) return EMIN_ERR_ARG;
  *out = nullptr;
  emin_matrix_t* h = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const emin_status st = guard([&] {
    check_csr_arg(M);
    check_csr_arg(P);
    if (M->nrows != M->ncols || P->nrows != M->nrows)
      throw Error(EMIN_ERR_SHAPE, "P^T M P: M must be square with P's row count");
    h = new emin_matrix_s();
    Arena& ar = h->ar;
    StreamUse use_ar(h->ar, s);
    int* derr = ar.alloc<int>(1);
    HIP_OK(hipMemsetAsync(derr, 0, sizeof(int), s));
    const CsrView Mv = viewof(*M), Pv = viewof(*P);
    validate_csr(Mv, false, derr, s);
    validate_csr(Pv, false, derr, s);
    if (d2h(derr, s)) throw Error(EMIN_ERR_PATTERN, "malformed CSR");
    Csr PT, T;
    int32_t* src = nullptr;
    transpose_pattern(Pv, PT, src, s, ar);
    PT.val = ar.alloc<double>(PT.nnz);
    gather_values(P->val, src, PT.val, PT.nnz, s);
    SpgemmPlan p1, p2;
    spgemm_symbolic(Mv, Pv, T, p1, s, ar, nullptr, true);
    spgemm_numeric(Mv, Pv, T, p1, s);
    spgemm_symbolic(view(PT), view(T), h->C, p2, s, ar, nullptr, true);
    spgemm_numeric(view(PT), view(T), h->C, p2, s);
    HIP_OK(hipStreamSynchronize(s));
  });
  if (st != EMIN_OK) {
    if (h) {
      (void)hipStreamSynchronize(s);
      delete h;
    }
    return st;
  }
  *out = h;
  return EMIN_OK;
}

emin_status emin_matrix_view(const emin_matrix_t* m, emin_csr_t* out) {
  if (!m || !out) return EMIN_ERR_ARG;
  *out = emin_csr_t{m->C.nrows, m->C.ncols, m->C.nnz, m->C.rowptr, m->C.col, m->C.val};
  return EMIN_OK;
}

void emin_matrix_destroy(emin_matrix_t* m) { delete m; }

emin_status emin_infsup(const emin_csr_t* B, const emin_csr_t* Mv, const emin_csr_t* Mp,
                        int32_t dim, int32_t steps, double rel, double* sigma_min,
                        double* resid, int32_t* nzero, int32_t* steps_done, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return guard([&] {
    check_csr_arg(B);
    check_csr_arg(Mv);
    check_csr_arg(Mp);
    if (!sigma_min) throw Error(EMIN_ERR_ARG, "NULL output");
    if (dim < 1 || dim > 3 || steps < 1 || !(rel >= 0.0)) throw Error(EMIN_ERR_ARG, "parameter");
    const int64_t np = B->nrows, nvd = B->ncols, nv = Mv->nrows;
    if (Mp->nrows != np || Mp->ncols != np || Mv->ncols != nv || nvd != dim * nv)
      throw Error(EMIN_ERR_SHAPE, "B must be n_p x d*n_v with M_p n_p x n_p, M_v n_v x n_v");
    const int m = (int)std::min<int64_t>(steps, np);
    Arena ar;
    StreamUse use_ar(ar, s);
    try {
      int* derr = ar.alloc<int>(1);
      HIP_OK(hipMemsetAsync(derr, 0, sizeof(int), s));
      const CsrView Bv = viewof(*B);
      validate_csr(Bv, true, derr, s);
      validate_csr(viewof(*Mv), true, derr, s);
      validate_csr(viewof(*Mp), true, derr, s);
      const int e = d2h(derr, s);
      if (e & DERR_PATTERN) throw Error(EMIN_ERR_PATTERN, "malformed CSR");
      if (e & DERR_VALUE) throw Error(EMIN_ERR_VALUE, "non-finite value");
      double* dv = ar.alloc<double>(nv);
      double* dp = ar.alloc<double>(np);
      if (nv) k_lump_abs<<<nblocks(nv, 256), 256, 0, s>>>(Mv->rowptr, Mv->val, nv, dv);
      if (np) k_lump_abs<<<nblocks(np, 256), 256, 0, s>>>(Mp->rowptr, Mp->val, np, dp);
      Csr BT;
      int32_t* src = nullptr;
      transpose_pattern(Bv, BT, src, s, ar);
      BT.val = ar.alloc<double>(BT.nnz);
      gather_values(B->val, src, BT.val, BT.nnz, s);
      double* Q = ar.alloc<double>((size_t)(m + 2) * (size_t)np);
      double* w = ar.alloc<double>(np);
      double* t1 = ar.alloc<double>(np);
      double* tv = ar.alloc<double>(nvd);
      double* c = ar.alloc<double>(m + 2);
      double* c2 = ar.alloc<double>(m + 2);
      double* alpha = ar.alloc<double>(m);
      double* beta = ar.alloc<double>(m);
      double* nrm = ar.alloc<double>(1);
      int* stop = ar.alloc<int>(2);
      double* ritz = ar.alloc<double>(4);
      double* rwk = ar.alloc<double>((size_t)5 * m);
      HIP_OK(hipMemsetAsync(stop, 0, 2 * sizeof(int), s));
      const unsigned gp = nblocks(np, 256);
      // w = S x = Dp^-1/2 B Dv^-1 B^T Dp^-1/2 x
      auto apply_S = [&](const double* x, double* out) {
        k_dscale<<<gp, 256, 0, s>>>(x, dp, np, np, 1, t1);
        k_spmv<<<nblocks(nvd, 256), 256, 0, s>>>(BT.rowptr, BT.col, BT.val, nvd, t1, tv);
        k_dscale<<<nblocks(nvd, 256), 256, 0, s>>>(tv, dv, nvd, nv, 2, tv);
        k_spmv<<<gp, 256, 0, s>>>(B->rowptr, B->col, B->val, np, tv, t1);
        k_dscale<<<gp, 256, 0, s>>>(t1, dp, np, np, 1, out);
      };
      auto dot1 = [&](const double* a, const double* b, double* res) {
        k_qt_dot<<<1, IB, 0, s>>>(a, b, np, res);
      };
      // The hydrostatic pressure of an enclosed flow (B^T 1 = 0) is the
      // null vector Dp^1/2 1 of S: when its Rayleigh quotient vanishes
      // against the start vector's, it is held as a locked first vector
      // (counted as one zero singular value) and Lanczos runs on its
      // complement, where the smallest eigenvalue is sigma_min^2.
      double* v0 = Q;
      double* q1 = Q + (int64_t)np;
      k_lump_abs<<<gp, 256, 0, s>>>(Mp->rowptr, Mp->val, np, v0);   // = dp
      k_dscale<<<gp, 256, 0, s>>>(v0, dp, np, np, 1, v0);             // dp / sqrt(dp)
      dot1(v0, v0, nrm);
      k_scale_by<<<gp, 256, 0, s>>>(v0, np, nrm);
      k_lz_start<<<gp, 256, 0, s>>>(np, q1);
      dot1(q1, q1, nrm);
      k_scale_by<<<gp, 256, 0, s>>>(q1, np, nrm);
      double rq[2];
      apply_S(v0, w);
      dot1(v0, w, c);
      apply_S(q1, w);
      dot1(q1, w, c + 1);
      HIP_OK(hipMemcpyAsync(rq, c, sizeof(rq), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      const int off = (np > 1 && std::fabs(rq[0]) <= 1e-12 * std::fabs(rq[1])) ? 1 : 0;
      const int mm = std::min<int>(m, (int)np - off);
      if (off) {
        // start vector orthogonal to the locked one
        k_qt_dot<<<1, IB, 0, s>>>(Q, q1, np, c);
        k_multi_axpy<<<gp, 256, 0, s>>>(Q, 1, c, np, q1);
        dot1(q1, q1, nrm);
        k_scale_by<<<gp, 256, 0, s>>>(q1, np, nrm);
      } else {
        HIP_OK(hipMemcpyAsync(v0, q1, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
      }
      int done = 0;
      for (int j = 0; j < mm; j++) {
        const int jq = off + j;                 // q_j's row in Q
        const double* qj = Q + (int64_t)jq * np;
        apply_S(qj, w);
        // re-orthogonalise against every earlier vector (the locked one
        // included), twice; alpha_j from the first pass
        k_qt_dot<<<jq + 1, IB, 0, s>>>(Q, w, np, c);
        k_multi_axpy<<<gp, 256, 0, s>>>(Q, jq + 1, c, np, w);
        k_qt_dot<<<jq + 1, IB, 0, s>>>(Q, w, np, c2);
        k_multi_axpy<<<gp, 256, 0, s>>>(Q, jq + 1, c2, np, w);
        dot1(w, w, nrm);
        k_lz_scalars<<<1, 64, 0, s>>>(c + off, j, nrm, alpha, beta, stop);
        k_lz_next<<<gp, 256, 0, s>>>(w, beta, j, stop, np, Q + (int64_t)(jq + 1) * np);
        done = j + 1;
        if ((j & 15) == 15 && d2h(stop, s)) break;   // invariant Krylov space: T is complete
      }
      (void)done;
      k_lz_ritz<<<1, 64, 0, s>>>(alpha, beta, stop + 1, rel * rel, rwk, ritz);
      double hr[4];
      int hs[2];
      HIP_OK(hipMemcpyAsync(hr, ritz, sizeof(hr), hipMemcpyDeviceToHost, s));
      HIP_OK(hipMemcpyAsync(hs, stop, sizeof(hs), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      *sigma_min = hr[2] > 0.0 ? std::sqrt(hr[2]) : 0.0;
      if (resid) *resid = hr[3];
      if (nzero) *nzero = (int32_t)hr[1] + off;
      if (steps_done) *steps_done = hs[1];
    } catch (...) {
      (void)hipStreamSynchronize(s);
      throw;
    }
  });
}

}  // extern "C"
