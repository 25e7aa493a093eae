// C ABI: one level of Alg. 1 as emin_pattern / emin_setup / emin_rap.
#include <cstring>
#include <memory>
#include <mutex>

#include "coarsen.h"
#include "emin_cg.h"

using namespace emin;

struct emin_pattern_s {
  Arena ar;
  // temporaries of the pattern build (released at its end, after its work)
  Scratch tmp;
  int dim = 2;
  int64_t n_v = 0, n_p = 0, nnzA = 0, nnzB = 0;
  int lds_max = 65536;
  // aux operators (eq. e:filtering) and energy operators
  Csr BT;
  int32_t* bt_src = nullptr;
  Csr Z;
  SpgemmPlan zplan;
  double *dZ = nullptr, *dA = nullptr;
  uint8_t *keep_p = nullptr, *keep_v = nullptr;
  Csr Atp, Atv, Mp, Mv;
  int32_t *mp_ia = nullptr, *mp_ib = nullptr, *mv_ia = nullptr, *mv_ib = nullptr;
  // EMIN_FLAG_ENERGY_ATA: the velocity energy operator A~^T A~ (Mv stays the
  // velocity graph)
  bool ata = false;
  // EMIN_FLAG_GMRES: the velocity block's operator is A~ itself, GMRES form
  bool gmres = false;
  GmresWork gv;
  // EMIN_FLAG_PETROV_GALERKIN: the restriction's operator A~ A~^T (CG form) or
  // A~^T (GMRES form), its workspace, and the Galerkin product's extra values
  bool pg = false;
  Csr Er;
  SpgemmPlan erplan;
  EminWork er;
  GmresWork gr;
  float* Mrf = nullptr;
  double *X2val = nullptr, *U2val = nullptr;
  Csr AtvT, Ev;
  int32_t* atvt_src = nullptr;
  SpgemmPlan evplan;
  float *Mpf = nullptr, *Mvf = nullptr;
  uint8_t* dir = nullptr;
  double* xp = nullptr;
  // coarsening and patterns
  CoarsenArgs ca;
  CoarsenOut cp;
  uint8_t* cbar = nullptr;
  int64_t n_mid = 0;
  uint8_t* cv = nullptr;
  VPatternOut vp;
  // EMIN
  EminWork ev, ep;
  double *Wv_def = nullptr, *Wp_def = nullptr;
  emin_report_t* rep_internal = nullptr;
  // Galerkin product
  Csr PvT, T, Ac, X, U, PpT, Bc;
  int32_t *pvt_src = nullptr, *x_src = nullptr, *ppt_src = nullptr;
  SpgemmPlan tplan, acplan, uplan, bcplan;
  // FP32 copies for the mixed-precision Galerkin product (allocated on first use)
  float *Af = nullptr, *Bf = nullptr, *Pvf = nullptr, *Ppf = nullptr, *PvTf = nullptr,
        *Xf = nullptr, *PpTf = nullptr, *Tf = nullptr, *Uf = nullptr;
  // coarse descriptors
  double* xv_c = nullptr;
  int32_t* p2v_c = nullptr;
  int* derr = nullptr;
  emin_sizes_t sizes{};
};

static thread_local std::string g_last_error;

void emin::set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

__global__ void k_zero_words(uint32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

void emin::zero_bytes(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n) k_zero_words<<<nblocks(n, 256), 256, 0, s>>>(static_cast<uint32_t*>(p), n);
}

namespace {

__global__ void k_fp_probe(const double* x, double* sq, double* rc, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  sq[i] = sqrt(x[i]);
  rc[i] = 1.0 / x[i];
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

CsrView in_view(const emin_csr_t& c) { return {c.nrows, c.ncols, c.nnz, c.rowptr, c.col, c.val}; }

__global__ void k_gather_coords(const double* xv, const int32_t* idx, int64_t n, int dim,
                                double* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int d = 0; d < dim; d++) out[i * dim + d] = xv[(int64_t)idx[i] * dim + d];
}

__global__ void k_check_idx(const int32_t* idx, int64_t n, int64_t bound, int* derr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (idx[i] < 0 || idx[i] >= bound)) atomicOr(derr, DERR_PATTERN);
}

// a C row (cid >= 0) holds exactly its own coarse column; cid < nc
__global__ void k_check_cid(const int32_t* cid, const int64_t* nrp, const int32_t* ncol,
                            int64_t n, int64_t nc, int* derr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t c = cid[i];
  if (c >= nc || (c >= 0 && (nrp[i + 1] - nrp[i] != 1 || ncol[nrp[i]] != c)))
    atomicOr(derr, DERR_PATTERN);
}

__global__ void k_cv_from_cbar(const uint8_t* cbar, const int32_t* p2v, int64_t n_p, uint8_t* cv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_p && cbar[i]) cv[p2v[i]] = 1;
}

__global__ void k_p2v_coarse(const int32_t* clist_p, const int32_t* p2v, const int32_t* cid_v,
                             int64_t n_pc, int32_t* out, int* derr) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_pc) return;
  const int32_t v = cid_v[p2v[clist_p[c]]];
  if (v < 0) atomicOr(derr, DERR_COLOCATE);
  out[c] = v;
}

// X = I_d (x) Pv: pattern and the map from X's entries to Pv's
// X = I_d (x) P: row c n + i of X is row i of P with its columns shifted by
// c nc; one thread per entry of X (and per row pointer)
__global__ void k_kron_entries(const int32_t* pcol, int64_t nnz, int64_t nc, int dim,
                               int32_t* xcol, int32_t* xsrc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dim * nnz) return;
  const int64_t c = e / nnz, e0 = e - c * nnz;
  xcol[e] = (int32_t)(c * nc + pcol[e0]);
  xsrc[e] = (int32_t)e0;
}

__global__ void k_kron_rowptr(const int64_t* prp, int64_t n, int64_t nnz, int dim, int64_t* xrp) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > dim * n) return;
  const int64_t c = r < dim * n ? r / n : dim - 1;
  const int64_t i = r < dim * n ? r - c * n : n;
  xrp[r] = c * nnz + prp[i];
}

void check_derr(emin_pattern_t* h, hipStream_t s) {
  const int e = d2h(h->derr, s);
  if (e & DERR_PATTERN) throw Error(EMIN_ERR_PATTERN, "malformed CSR or index array");
  if (e & DERR_VALUE) throw Error(EMIN_ERR_VALUE, "non-finite input value");
  if (e & DERR_CAPACITY) throw Error(EMIN_ERR_CAPACITY, "capacity exceeded");
  if (e & DERR_COLOCATE) throw Error(EMIN_ERR_COLOCATE, "coarse pressure without coarse velocity");
}

void check_system(const emin_system_t* sys) {
  if (!sys) throw Error(EMIN_ERR_ARG, "NULL system");
  if (sys->dim < 2 || sys->dim > 3) throw Error(EMIN_ERR_ARG, "dim must be 2 or 3");
  const emin_csr_t& A = sys->Ahat;
  const emin_csr_t& B = sys->Bdiv;
  if (A.nrows < 0 || A.nnz < 0 || B.nrows < 0 || B.nnz < 0) throw Error(EMIN_ERR_ARG, "negative size");
  if (A.nrows != A.ncols) throw Error(EMIN_ERR_SHAPE, "Ahat must be square");
  if (B.ncols != sys->dim * A.nrows) throw Error(EMIN_ERR_SHAPE, "Bdiv must have dim*n_v columns");
  if ((A.nrows && (!A.rowptr || (A.nnz && (!A.col || !A.val)))) ||
      (B.nrows && (!B.rowptr || (B.nnz && (!B.col || !B.val)))) ||
      (A.nrows && !sys->xv) || (B.nrows && !sys->p2v))
    throw Error(EMIN_ERR_ARG, "NULL array");
  if (A.nnz >= INT32_MAX || B.nnz >= INT32_MAX) throw Error(EMIN_ERR_CAPACITY, "nnz >= 2^31");
}

void check_params(const emin_params_t* p) {
  if (!p) throw Error(EMIN_ERR_ARG, "NULL params");
  if (p->iters < 0 || p->iters > EMIN_MAX_ITERS) throw Error(EMIN_ERR_ARG, "iters out of range");
  if (!(p->tau1_v >= 0.0) || !(p->tau1_p >= 0.0) || !(p->tau2_sq >= 0.0))
    throw Error(EMIN_ERR_ARG, "negative tolerance");
  if (p->precision != EMIN_PREC_F64 && p->precision != EMIN_PREC_MIXED)
    throw Error(EMIN_ERR_ARG, "unknown precision");
}

int pick_lanes(const Csr& M) {
  const double avg = M.nrows ? (double)M.nnz / (double)M.nrows : 1.0;
  int g = 4;
  while (g < 64 && 2 * g < avg) g <<= 1;
  return g;
}

// the operator of the velocity block's EMIN: A~^T A~ (A^T A-norm), A~ itself
// (GMRES form) or the symmetric part (A-norm)
static const Csr& energy_v(const emin_pattern_t* h) {
  return h->ata ? h->Ev : (h->gmres ? h->Atv : h->Mv);
}

// the restriction's operator (Petrov-Galerkin): A~ A~^T, or A~^T (GMRES form)
static const Csr& energy_r(const emin_pattern_t* h) { return h->gmres ? h->AtvT : h->Er; }

// A~^T's values, then E = A~^T A~ and the restriction's A~ A~^T from the
// filtered operator's current values
static void ata_numeric(emin_pattern_t* h, hipStream_t s) {
  gather_values(h->Atv.val, h->atvt_src, h->AtvT.val, h->AtvT.nnz, s);
  if (h->ata) spgemm_numeric(view(h->AtvT), view(h->Atv), h->Ev, h->evplan, s);
  if (h->pg && !h->gmres) spgemm_numeric(view(h->Atv), view(h->AtvT), h->Er, h->erplan, s);
}

// A second stream (default priority, non-blocking) and two events per host
// thread and device, for work of a pattern build that runs beside the main
// stream's; kept until the process ends.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

SideStream& side_stream() {
  thread_local SideStream per_dev[64];
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(EMIN_ERR_DEVICE, "device index");
  SideStream& x = per_dev[dev];
  if (!x.s) {
    HIP_OK(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&x.join, hipEventDisableTiming));
  }
  return x;
}

void build_pattern(emin_pattern_t* h, const emin_system_t* sys, const emin_params_t* prm,
                   hipStream_t s, const int32_t* cp_given = nullptr, int64_t ncp = 0) {
  Arena& ar = h->ar;
  StreamUse use_ar(h->ar, s), use_tmp(h->tmp.ar, s);
  const int dim = sys->dim;
  const int64_t nv = sys->Ahat.nrows, np = sys->Bdiv.nrows;
  h->dim = dim;
  h->n_v = nv;
  h->n_p = np;
  h->nnzA = sys->Ahat.nnz;
  h->nnzB = sys->Bdiv.nnz;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&h->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  h->derr = ar.alloc<int>(1);
  HIP_OK(hipMemsetAsync(h->derr, 0, sizeof(int), s));
  const CsrView A = in_view(sys->Ahat), B = in_view(sys->Bdiv);
  const bool vals = (prm->flags & EMIN_FLAG_VALIDATE) != 0;
  h->ata = (prm->flags & EMIN_FLAG_ENERGY_ATA) != 0;
  h->gmres = (prm->flags & EMIN_FLAG_GMRES) != 0;
  if (h->ata && h->gmres)
    throw Error(EMIN_ERR_ARG, "EMIN_FLAG_GMRES takes A~ itself, not the A^T A operator");
  h->pg = (prm->flags & EMIN_FLAG_PETROV_GALERKIN) != 0;
  validate_csr(A, vals, h->derr, s);
  validate_csr(B, vals, h->derr, s);
  if (np) k_check_idx<<<nblocks(np, 256), 256, 0, s>>>(sys->p2v, np, nv, h->derr);
  check_derr(h, s);
  // (the side stream's work below needs only the validated inputs)
  SideStream& side = side_stream();
  HIP_OK(hipEventRecord(side.fork, s));

  // pressure coordinates: those of the co-located velocity nodes
  h->xp = ar.alloc<double>((size_t)np * dim);
  if (np) k_gather_coords<<<nblocks(np, 256), 256, 0, s>>>(sys->xv, sys->p2v, np, dim, h->xp);

  // form_aux_block_diagonal: Z = B B^T, filtered; filtered velocity block
  transpose_pattern(B, h->BT, h->bt_src, s, ar);
  h->BT.val = ar.alloc<double>(h->BT.nnz);
  gather_values(B.val, h->bt_src, h->BT.val, h->BT.nnz, s);
  spgemm_symbolic(B, view(h->BT), h->Z, h->zplan, s, ar, h->derr, false, &h->tmp);
  spgemm_numeric_aat(B, view(h->BT), h->Z, h->zplan, s);
  h->dZ = ar.alloc<double>(np);
  diag_of(view(h->Z), h->dZ, s);
  h->keep_p = ar.alloc<uint8_t>(h->Z.nnz);
  filter_symbolic(view(h->Z), prm->tau1_p, h->dZ, h->keep_p, h->Atp, s, ar);
  symmetrize_symbolic(h->Atp, h->Mp, h->mp_ia, h->mp_ib, s, ar);
  symmetrize_numeric(h->Atp.val, h->mp_ia, h->mp_ib, h->Mp, s);
  // the filtered velocity block, its energy operator and the Dirichlet rows
  // do not depend on Alg. 3: they are queued on a side stream while the
  // single-workgroup kernels of Alg. 3 run
  auto velocity_filter = [&]() {
    hipStream_t s2 = side.s;
    try {
      HIP_OK(hipStreamWaitEvent(s2, side.fork, 0));
      h->dA = ar.alloc<double>(nv);
      diag_of(A, h->dA, s2);
      h->keep_v = ar.alloc<uint8_t>(A.nnz);
      h->dir = ar.alloc<uint8_t>(nv);
      // (the Dirichlet flags come from the filter's count pass)
      filter_symbolic(A, prm->tau1_v, h->dA, h->keep_v, h->Atv, s2, ar, h->dir);
      symmetrize_symbolic(h->Atv, h->Mv, h->mv_ia, h->mv_ib, s2, ar);
      symmetrize_numeric(h->Atv.val, h->mv_ia, h->mv_ib, h->Mv, s2);
      HIP_OK(hipEventRecord(side.join, s2));
      HIP_OK(hipStreamWaitEvent(s, side.join, 0));
    } catch (...) {
      // nothing queued on the side stream may outlive the handle's memory
      (void)hipStreamSynchronize(s2);
      throw;
    }
  };

  // Alg. 3 + extra distance-3 points on the graph of the pressure operator
  h->ca.grp = h->Mp.rowptr;
  h->ca.gcol = h->Mp.col;
  h->ca.n = np;
  h->ca.dim = dim;
  h->ca.x = h->xp;
  bool filtered = false;
  coarsen_pressure(h->ca, h->cp, s, ar, h->lds_max, cp_given, ncp, [&]() {
    velocity_filter();
    filtered = true;
  });
  if (!filtered) velocity_filter();

  // sec. 4.3, eq. (min_problem): the A^T A-norm for a non-symmetric block
  if (h->ata || h->pg) {
    transpose_pattern(view(h->Atv), h->AtvT, h->atvt_src, s, ar);
    h->AtvT.val = ar.alloc<double>(h->AtvT.nnz);
    if (h->ata)
      spgemm_symbolic(view(h->AtvT), view(h->Atv), h->Ev, h->evplan, s, ar, h->derr, false,
                      &h->tmp);
    if (h->pg && !h->gmres)
      spgemm_symbolic(view(h->Atv), view(h->AtvT), h->Er, h->erplan, s, ar, h->derr, false,
                      &h->tmp);
    ata_numeric(h, s);
  }

  // Alg. 4 mid-points, co-located velocities, velocity pattern
  h->cbar = ar.alloc<uint8_t>(np);
  const int64_t ncbar = midpoints(h->cp.S, h->ca.st, h->xp, dim, prm->tau2_sq, h->cbar, s, ar,
                                  h->lds_max);
  h->n_mid = ncbar - h->cp.n_c;
  h->cv = ar.alloc<uint8_t>(nv);
  HIP_OK(hipMemsetAsync(h->cv, 0, nv, s));
  if (np) k_cv_from_cbar<<<nblocks(np, 256), 256, 0, s>>>(h->cbar, sys->p2v, np, h->cv);
  velocity_pattern(h->Mv, h->dir, h->cv, h->vp, s, ar, h->lds_max);

  // EMIN workspace
  const bool mixed = true;  // FP32 copies are allocated so either mode can run
  h->ev.allocate(nv, h->vp.N.nnz, h->vp.n_c, ar, mixed);
  h->ep.allocate(np, h->cp.N.nnz, h->cp.n_c, ar, mixed);
  h->ev.g = pick_lanes(energy_v(h));
  h->ep.g = pick_lanes(h->Mp);
  h->ev.smax = (int)max_row_len(h->vp.N.rowptr, nv, s, ar);
  h->ep.smax = (int)max_row_len(h->cp.N.rowptr, np, s, ar);
  if (h->ev.smax > 64 || h->ep.smax > 64) throw Error(EMIN_ERR_CAPACITY, "pattern row > 64");
  const bool tune = (prm->flags & EMIN_FLAG_AUTOTUNE) != 0;
  const bool stage = (prm->flags & EMIN_FLAG_STAGED_PRODUCT) != 0;
  // (tiles of the velocity rows by their coordinates, of the pressure rows by
  // their co-located velocity nodes')
  h->ev.make_bins(energy_v(h), h->vp.N.rowptr, h->vp.N.col, s, ar, tune, stage, sys->xv, nullptr,
                  dim);
  h->ep.make_bins(h->Mp, h->cp.N.rowptr, h->cp.N.col, s, ar, tune, stage, sys->xv, sys->p2v, dim);
  if (h->pg) {
    h->er.allocate(nv, h->vp.N.nnz, h->vp.n_c, ar, mixed);
    h->er.g = pick_lanes(energy_r(h));
    h->er.smax = h->ev.smax;
    h->er.make_bins(energy_r(h), h->vp.N.rowptr, h->vp.N.col, s, ar, tune, stage, sys->xv,
                    nullptr, dim);
    h->Mrf = ar.alloc<float>(energy_r(h).nnz);
  }
  h->Mvf = ar.alloc<float>(energy_v(h).nnz);
  h->Mpf = ar.alloc<float>(h->Mp.nnz);
  h->Wv_def = ar.alloc<double>(nv);
  h->Wp_def = ar.alloc<double>(np);
  default_modes(h->dir, nv, h->Wv_def, s);
  default_modes(nullptr, np, h->Wp_def, s);
  h->rep_internal = ar.alloc<emin_report_t>(1);

  // Galerkin product, symbolic: Ac = Pv^T (Ahat Pv), Bc = Pp^T (Bdiv (I_d (x) Pv))
  Csr Pv = h->vp.N, Pp = h->cp.N;
  transpose_pattern(view(Pv), h->PvT, h->pvt_src, s, ar);
  h->PvT.val = ar.alloc<double>(h->PvT.nnz);
  spgemm_symbolic(A, view(Pv), h->T, h->tplan, s, ar, h->derr, true, &h->tmp);
  spgemm_symbolic(view(h->PvT), view(h->T), h->Ac, h->acplan, s, ar, h->derr, true, &h->tmp);
  h->X.nrows = (int64_t)dim * nv;
  h->X.ncols = (int64_t)dim * h->vp.n_c;
  h->X.nnz = (int64_t)dim * Pv.nnz;
  h->X.rowptr = ar.alloc<int64_t>(h->X.nrows + 1);
  h->X.col = ar.alloc<int32_t>(h->X.nnz);
  h->X.val = ar.alloc<double>(h->X.nnz);
  h->x_src = ar.alloc<int32_t>(h->X.nnz);
  if (nv) {
    k_kron_rowptr<<<nblocks(h->X.nrows + 1, 256), 256, 0, s>>>(Pv.rowptr, nv, Pv.nnz, dim,
                                                                h->X.rowptr);
    if (h->X.nnz)
      k_kron_entries<<<nblocks(h->X.nnz, 256), 256, 0, s>>>(Pv.col, Pv.nnz, h->vp.n_c, dim,
                                                             h->X.col, h->x_src);
  } else {
    HIP_OK(hipMemsetAsync(h->X.rowptr, 0, sizeof(int64_t), s));
  }
  spgemm_symbolic(B, view(h->X), h->U, h->uplan, s, ar, h->derr, true, &h->tmp);
  transpose_pattern(view(Pp), h->PpT, h->ppt_src, s, ar);
  h->PpT.val = ar.alloc<double>(h->PpT.nnz);
  spgemm_symbolic(view(h->PpT), view(h->U), h->Bc, h->bcplan, s, ar, h->derr, true, &h->tmp);

  // coarse descriptors: coordinates by injection, co-location map
  h->xv_c = ar.alloc<double>((size_t)h->vp.n_c * dim);
  if (h->vp.n_c)
    k_gather_coords<<<nblocks(h->vp.n_c, 256), 256, 0, s>>>(sys->xv, h->vp.clist, h->vp.n_c, dim,
                                                             h->xv_c);
  h->p2v_c = ar.alloc<int32_t>(h->cp.n_c);
  if (h->cp.n_c)
    k_p2v_coarse<<<nblocks(h->cp.n_c, 256), 256, 0, s>>>(h->cp.clist, sys->p2v, h->vp.cid,
                                                          h->cp.n_c, h->p2v_c, h->derr);
  check_derr(h, s);
  HIP_OK(hipStreamSynchronize(s));
  h->tmp.release();

  emin_sizes_t& z = h->sizes;
  z.n_v = nv;
  z.n_p = np;
  z.n_vc = h->vp.n_c;
  z.n_pc = h->cp.n_c;
  z.n_cp_alg3 = h->cp.n_alg3;
  z.n_cp_extra = h->cp.n_c - h->cp.n_alg3;
  z.n_mid = h->n_mid;
  z.n_cv_extra = h->vp.n_extra;
  z.nnz_Pv = h->vp.N.nnz;
  z.nnz_Pp = h->cp.N.nnz;
  z.nnz_Mv = energy_v(h).nnz;
  z.nnz_Mp = h->Mp.nnz;
  z.nnz_Ac = h->Ac.nnz;
  z.nnz_Bc = h->Bc.nnz;
  z.device_bytes = (int64_t)ar.bytes();
  z.sched_v = h->ev.sched_code();
  z.sched_p = h->ep.sched_code();
}

void check_same_structure(const emin_pattern_t* h, const emin_system_t* sys) {
  check_system(sys);
  if (sys->dim != h->dim || sys->Ahat.nrows != h->n_v || sys->Bdiv.nrows != h->n_p ||
      sys->Ahat.nnz != h->nnzA || sys->Bdiv.nnz != h->nnzB)
    throw Error(EMIN_ERR_SHAPE, "system structure differs from the pattern's");
}

void run_setup(emin_pattern_t* h, const emin_system_t* sys, const emin_params_t* prm, double* Pv,
               double* Pp, hipStream_t s, emin_report_t* rep, double* Rvt = nullptr) {
  StreamUse use_ar(h->ar, s);
  check_same_structure(h, sys);
  check_params(prm);
  if (((prm->flags & EMIN_FLAG_ENERGY_ATA) != 0) != h->ata)
    throw Error(EMIN_ERR_ARG, "energy norm differs from the pattern's (EMIN_FLAG_ENERGY_ATA)");
  if (((prm->flags & EMIN_FLAG_GMRES) != 0) != h->gmres)
    throw Error(EMIN_ERR_ARG, "solver form differs from the pattern's (EMIN_FLAG_GMRES)");
  if (((prm->flags & EMIN_FLAG_PETROV_GALERKIN) != 0) != h->pg)
    throw Error(EMIN_ERR_ARG, "restriction differs from the pattern's (EMIN_FLAG_PETROV_GALERKIN)");
  if ((h->sizes.nnz_Pv && !Pv) || (h->sizes.nnz_Pp && !Pp)) throw Error(EMIN_ERR_ARG, "NULL P");
  const CsrView A = in_view(sys->Ahat), B = in_view(sys->Bdiv);
  emin_report_t* r = rep ? rep : h->rep_internal;
  // a kernel, not a memset node: this path may be captured into a graph
  zero_bytes(r, sizeof(emin_report_t), s);
  // energy operators on the stored drop masks (emin_pattern formed them
  // already from values the caller vouches are unchanged)
  if ((prm->flags & EMIN_FLAG_PATTERN_VALUES) == 0) {
    gather_values(B.val, h->bt_src, h->BT.val, h->BT.nnz, s);
    spgemm_numeric_aat(B, view(h->BT), h->Z, h->zplan, s);
    diag_of(view(h->Z), h->dZ, s);
    filter_numeric(view(h->Z), h->keep_p, h->dZ, h->Atp, s);
    symmetrize_numeric(h->Atp.val, h->mp_ia, h->mp_ib, h->Mp, s);
    diag_of(A, h->dA, s);
    filter_numeric(A, h->keep_v, h->dA, h->Atv, s);
    symmetrize_numeric(h->Atv.val, h->mv_ia, h->mv_ib, h->Mv, s);
    if (h->ata || h->pg) ata_numeric(h, s);
  }
  const bool mixed = prm->precision == EMIN_PREC_MIXED;
  if (mixed) {
    to_float(energy_v(h).val, h->Mvf, energy_v(h).nnz, s);
    to_float(h->Mp.val, h->Mpf, h->Mp.nnz, s);
  }
  const bool energy = (prm->flags & EMIN_FLAG_ENERGY) != 0;
  EminReportPtrs rv{r->energy_v, r->rho_v, r->gamma_v, &r->its_v, &r->status};
  EminReportPtrs rpp{r->energy_p, r->rho_p, r->gamma_p, &r->its_p, &r->status};
  const double* Wv = sys->Wv ? sys->Wv : h->Wv_def;
  const double* Wp = sys->Wp ? sys->Wp : h->Wp_def;
  if (h->gmres) {
    h->gv.reserve(prm->iters, h->vp.N.nnz, 0, h->ar);
    run_emin_gmres(h->ev, energy_v(h), h->Mvf, h->vp.N.rowptr, h->vp.N.col, h->vp.cid,
                   h->vp.clist, Wv, Pv, prm->iters, mixed, rv, h->gv, s);
  } else {
    run_emin(h->ev, energy_v(h), h->Mvf, h->vp.N.rowptr, h->vp.N.col, h->vp.cid, h->vp.clist, Wv,
             Pv, prm->iters, energy, mixed, rv, s);
  }
  run_emin(h->ep, h->Mp, h->Mpf, h->cp.N.rowptr, h->cp.N.col, h->cp.cid, h->cp.clist, Wp, Pp,
           prm->iters, energy, mixed, rpp, s);
  if (Rvt) {
    // the Petrov-Galerkin restriction: R_v^T on the velocity pattern
    if (mixed) to_float(energy_r(h).val, h->Mrf, energy_r(h).nnz, s);
    EminReportPtrs rr{r->energy_r, r->rho_r, r->gamma_r, &r->its_r, &r->status};
    if (h->gmres) {
      h->gr.reserve(prm->iters, h->vp.N.nnz, 0, h->ar);
      run_emin_gmres(h->er, energy_r(h), h->Mrf, h->vp.N.rowptr, h->vp.N.col, h->vp.cid,
                     h->vp.clist, Wv, Rvt, prm->iters, mixed, rr, h->gr, s);
    } else {
      run_emin(h->er, energy_r(h), h->Mrf, h->vp.N.rowptr, h->vp.N.col, h->vp.cid, h->vp.clist,
               Wv, Rvt, prm->iters, energy, mixed, rr, s);
    }
  }
  HIP_OK(hipGetLastError());
}

void run_rap(emin_pattern_t* h, const emin_system_t* sys, const double* Pv, const double* Pp,
             double* Acv, double* Bcv, int precision, hipStream_t s) {
  StreamUse use_ar(h->ar, s);
  check_same_structure(h, sys);
  if (precision != EMIN_PREC_F64 && precision != EMIN_PREC_MIXED)
    throw Error(EMIN_ERR_ARG, "unknown precision");
  if ((h->sizes.nnz_Pv && !Pv) || (h->sizes.nnz_Pp && !Pp) || (h->Ac.nnz && !Acv) ||
      (h->Bc.nnz && !Bcv))
    throw Error(EMIN_ERR_ARG, "NULL value array");
  const CsrView A = in_view(sys->Ahat), B = in_view(sys->Bdiv);
  CsrView PvV{h->vp.N.nrows, h->vp.N.ncols, h->vp.N.nnz, h->vp.N.rowptr, h->vp.N.col, Pv};
  if (precision == EMIN_PREC_MIXED) {
    Arena& ar = h->ar;
    if (!h->Af) {
      h->Af = ar.alloc<float>(A.nnz);
      h->Bf = ar.alloc<float>(B.nnz);
      h->Pvf = ar.alloc<float>(h->vp.N.nnz);
      h->Ppf = ar.alloc<float>(h->cp.N.nnz);
      h->PvTf = ar.alloc<float>(h->PvT.nnz);
      h->Xf = ar.alloc<float>(h->X.nnz);
      h->PpTf = ar.alloc<float>(h->PpT.nnz);
      h->Tf = ar.alloc<float>(h->T.nnz);
      h->Uf = ar.alloc<float>(h->U.nnz);
    }
    to_float(A.val, h->Af, A.nnz, s);
    to_float(B.val, h->Bf, B.nnz, s);
    to_float(Pv, h->Pvf, h->vp.N.nnz, s);
    to_float(Pp, h->Ppf, h->cp.N.nnz, s);
    gather_values_f(h->Pvf, h->pvt_src, h->PvTf, h->PvT.nnz, s);
    gather_values_f(h->Pvf, h->x_src, h->Xf, h->X.nnz, s);
    gather_values_f(h->Ppf, h->ppt_src, h->PpTf, h->PpT.nnz, s);
    spgemm_numeric_f32(A, h->Af, PvV, h->Pvf, h->T, h->Tf, nullptr, h->tplan, s);
    spgemm_numeric_f32(view(h->PvT), h->PvTf, view(h->T), h->Tf, h->Ac, nullptr, Acv, h->acplan, s);
    spgemm_numeric_f32(B, h->Bf, view(h->X), h->Xf, h->U, h->Uf, nullptr, h->uplan, s);
    spgemm_numeric_f32(view(h->PpT), h->PpTf, view(h->U), h->Uf, h->Bc, nullptr, Bcv, h->bcplan, s);
    HIP_OK(hipGetLastError());
    return;
  }
  gather_values(Pv, h->pvt_src, h->PvT.val, h->PvT.nnz, s);
  spgemm_numeric(A, PvV, h->T, h->tplan, s);
  Csr Ac = h->Ac;
  Ac.val = Acv;
  spgemm_numeric(view(h->PvT), view(h->T), Ac, h->acplan, s);
  gather_values(Pv, h->x_src, h->X.val, h->X.nnz, s);
  spgemm_numeric(B, view(h->X), h->U, h->uplan, s);
  gather_values(Pp, h->ppt_src, h->PpT.val, h->PpT.nnz, s);
  Csr Bc = h->Bc;
  Bc.val = Bcv;
  spgemm_numeric(view(h->PpT), view(h->U), Bc, h->bcplan, s);
  HIP_OK(hipGetLastError());
}

// EMIN on one block with the energy operator, pattern, C rows and modes given
// (sec. 4.3, eq. (min_problem)); synchronous, with its own workspace.
void run_setup_with_pattern(const emin_csr_t* Min, const int64_t* nrp, const int32_t* ncol,
                            int64_t nc, int64_t nnz, const int32_t* cid, const double* W,
                            const double* Wc, int32_t iters, int32_t precision, uint32_t flags,
                            double* P, hipStream_t s, emin_report_t* rep,
                            Arena* ext = nullptr) {
  if (!Min) throw Error(EMIN_ERR_ARG, "NULL operator");
  const int64_t n = Min->nrows;
  if (n < 0 || nc < 0 || nnz < 0 || Min->nnz < 0) throw Error(EMIN_ERR_ARG, "negative size");
  if (Min->ncols != n) throw Error(EMIN_ERR_SHAPE, "operator must be square");
  if (iters < 0 || iters > EMIN_MAX_ITERS) throw Error(EMIN_ERR_ARG, "iters out of range");
  if (precision != EMIN_PREC_F64 && precision != EMIN_PREC_MIXED)
    throw Error(EMIN_ERR_ARG, "unknown precision");
  if (n && (!Min->rowptr || !nrp || !cid || !W || (Min->nnz && (!Min->col || !Min->val)) ||
            (nnz && (!ncol || !P)) || (nc && !Wc)))
    throw Error(EMIN_ERR_ARG, "NULL array");
  if (Min->nnz >= INT32_MAX || nnz >= INT32_MAX) throw Error(EMIN_ERR_CAPACITY, "nnz >= 2^31");
  Arena own;
  StreamUse use_own(own, s);
  Arena& ar = ext ? *ext : own;
  int* derr = ar.alloc<int>(1);
  HIP_OK(hipMemsetAsync(derr, 0, sizeof(int), s));
  const CsrView Mv = in_view(*Min);
  const CsrView Nv{n, nc, nnz, nrp, ncol, nullptr};
  validate_csr(Mv, (flags & EMIN_FLAG_VALIDATE) != 0, derr, s);
  validate_csr(Nv, false, derr, s);
  if (n) k_check_cid<<<nblocks(n, 256), 256, 0, s>>>(cid, nrp, ncol, n, nc, derr);
  const int e = d2h(derr, s);
  if (e & DERR_PATTERN) throw Error(EMIN_ERR_PATTERN, "malformed CSR or C rows");
  if (e & DERR_VALUE) throw Error(EMIN_ERR_VALUE, "non-finite input value");
  Csr M;
  M.nrows = n;
  M.ncols = n;
  M.nnz = Min->nnz;
  M.rowptr = const_cast<int64_t*>(Min->rowptr);
  M.col = const_cast<int32_t*>(Min->col);
  M.val = const_cast<double*>(Min->val);
  EminWork w;
  w.allocate(n, nnz, nc, ar, true);
  w.g = pick_lanes(M);
  w.smax = (int)max_row_len(nrp, n, s, ar);
  if (w.smax > 64) throw Error(EMIN_ERR_CAPACITY, "pattern row > 64");
  w.make_bins(M, nrp, ncol, s, ar, false, (flags & EMIN_FLAG_STAGED_PRODUCT) != 0);
  if (nc) HIP_OK(hipMemcpyAsync(w.Wc, Wc, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
  const bool mixed = precision == EMIN_PREC_MIXED;
  float* Mf = ar.alloc<float>(M.nnz);
  if (mixed) to_float(M.val, Mf, M.nnz, s);
  emin_report_t* r = rep ? rep : ar.alloc<emin_report_t>(1);
  zero_bytes(r, sizeof(emin_report_t), s);
  EminReportPtrs rp{r->energy_v, r->rho_v, r->gamma_v, &r->its_v, &r->status};
  run_emin(w, M, Mf, nrp, ncol, cid, nullptr, W, P, iters, (flags & EMIN_FLAG_ENERGY) != 0,
           mixed, rp, s);
  HIP_OK(hipGetLastError());
  // the workspace is released on return: wait for the kernels that use it
  HIP_OK(hipStreamSynchronize(s));
}

// Petrov-Galerkin coarse blocks (FP64): Ac = Rvt^T Ahat Pv, Bc = Pp^T Bdiv
// (I (x) Pv), Gct = Pp^T Gt (I (x) Rvt) on Bc's pattern (Gt: sys->Gt on Bdiv's
// pattern, or Bdiv itself)
void run_rap_pg(emin_pattern_t* h, const emin_system_t* sys, const double* Pv, const double* Pp,
                const double* Rvt, double* Acv, double* Bcv, double* Gctv, hipStream_t s) {
  StreamUse use_ar(h->ar, s);
  check_same_structure(h, sys);
  if (!h->pg) throw Error(EMIN_ERR_ARG, "pattern built without EMIN_FLAG_PETROV_GALERKIN");
  if ((h->sizes.nnz_Pv && (!Pv || !Rvt)) || (h->sizes.nnz_Pp && !Pp) || (h->Ac.nnz && !Acv) ||
      (h->Bc.nnz && (!Bcv || !Gctv)))
    throw Error(EMIN_ERR_ARG, "NULL value array");
  const CsrView A = in_view(sys->Ahat), B = in_view(sys->Bdiv);
  CsrView PvV{h->vp.N.nrows, h->vp.N.ncols, h->vp.N.nnz, h->vp.N.rowptr, h->vp.N.col, Pv};
  // Ac with R_v = Rvt^T: the transposed pattern carries Rvt's values
  gather_values(Rvt, h->pvt_src, h->PvT.val, h->PvT.nnz, s);
  spgemm_numeric(A, PvV, h->T, h->tplan, s);
  Csr Ac = h->Ac;
  Ac.val = Acv;
  spgemm_numeric(view(h->PvT), view(h->T), Ac, h->acplan, s);
  // Bc with P: the divergence block as in the Galerkin case
  gather_values(Pv, h->x_src, h->X.val, h->X.nnz, s);
  spgemm_numeric(B, view(h->X), h->U, h->uplan, s);
  gather_values(Pp, h->ppt_src, h->PpT.val, h->PpT.nnz, s);
  Csr Bc = h->Bc;
  Bc.val = Bcv;
  spgemm_numeric(view(h->PpT), view(h->U), Bc, h->bcplan, s);
  // Gct: the same products with (Gt, Rvt) in place of (Bdiv, Pv)
  if (!h->X2val) {
    h->X2val = h->ar.alloc<double>(h->X.nnz);
    h->U2val = h->ar.alloc<double>(h->U.nnz);
  }
  Csr X2 = h->X;
  X2.val = h->X2val;
  gather_values(Rvt, h->x_src, X2.val, X2.nnz, s);
  CsrView G = B;
  if (sys->Gt) G.val = sys->Gt;
  Csr U2 = h->U;
  U2.val = h->U2val;
  spgemm_numeric(G, view(X2), U2, h->uplan, s);
  Csr Gc = h->Bc;
  Gc.val = Gctv;
  spgemm_numeric(view(h->PpT), view(U2), Gc, h->bcplan, s);
  HIP_OK(hipGetLastError());
}

template <class F>
emin_status guarded(F&& f) {
  try {
    f();
    return EMIN_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    return EMIN_ERR_OOM;
  } catch (...) {
    return EMIN_ERR_DEVICE;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// The allocation-free variant of emin_setup_with_pattern: its workspace is a
// fixed device array of this file, one copy per GPU, reached through the
// address hipGetSymbolAddress returns for the current device (host code never
// passes the array's name to a kernel).
// ---------------------------------------------------------------------------
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static void* scratch_ptr() {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(EMIN_ERR_DEVICE, "device index");
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[dev] = p;
  }
  return ptr[dev];
}

// an upper bound of the workspace emin_setup_with_pattern takes (every
// array rounded up to 256 bytes, as the bump allocator does)
static size_t setup_with_pattern_bytes(int64_t n, int64_t nc, int64_t nnz, int64_t nnzm,
                                       int64_t smax) {
  auto r = [](double b) { return (size_t)((b + 255.0) / 256.0) * 256; };
  const int np = smax <= 8 ? 1 : (smax <= 16 ? 2 : 4);
  const double nb = (double)((n + 255) / 256);
  size_t b = 0;
  b += r(4) * 8;                                        // flags, scalars, small maxima
  b += r(8.0 * n) * 4 + r(8.0 * nc);                    // G, Wdef, rowdot, sched rows (+Wc)
  b += r(8.0 * nnz) * 4 + r(4.0 * nnz) * 2;             // R, Z, Q, MP; FP32 Z, Q
  b += r(8.0 * (2.0 * ((n + 3) / 4) + 16 + 8 * 9)) * 2; // block partials
  b += r(4.0 * nnzm) * (2 + np) + r((double)n);         // maps, FP32 M, eligibility
  b += r(8.0 * 9 * nb) * 2 + r(4.0 * ((n + 7) / 8 * 8 + 64));   // schedule counts, block map
  b += r(sizeof(emin_report_t)) + r(8.0 * 64) * 8;      // report, scan partials
  return b + (size_t(1) << 20);                         // slack for small arrays
}

extern "C" {

emin_status emin_pattern(const emin_system_t* sys, const emin_params_t* prm, void* stream,
                         emin_pattern_t** out) {
  if (!out) return EMIN_ERR_ARG;
  *out = nullptr;
  emin_pattern_t* h = nullptr;
  emin_status st = guarded([&] {
    check_system(sys);
    check_params(prm);
    h = new emin_pattern_s();
    build_pattern(h, sys, prm, as_stream(stream));
  });
  if (st != EMIN_OK) {
    if (h) {
      (void)hipStreamSynchronize(as_stream(stream));
      delete h;
    }
    return st;
  }
  set_last_error("");
  *out = h;
  return EMIN_OK;
}

emin_status emin_pattern_alloc(const emin_system_t* sys, const emin_params_t* prm,
                               const emin_allocator_t* alloc, void* stream, emin_pattern_t** out) {
  if (!out) return EMIN_ERR_ARG;
  *out = nullptr;
  emin_pattern_t* h = nullptr;
  emin_status st = guarded([&] {
    check_system(sys);
    check_params(prm);
    h = new emin_pattern_s();
    if (alloc) {
      h->ar.use_allocator(*alloc);
      h->tmp.ar.use_allocator(*alloc);
    }
    build_pattern(h, sys, prm, as_stream(stream));
  });
  if (st != EMIN_OK) {
    if (h) {
      // the queued work that uses the handle's blocks ends before they go back
      (void)hipStreamSynchronize(as_stream(stream));
      delete h;
    }
    return st;
  }
  set_last_error("");
  *out = h;
  return EMIN_OK;
}

emin_status emin_pattern_with_cpoints(const emin_system_t* sys, const emin_params_t* prm,
                                      const int32_t* cp, int64_t ncp, void* stream,
                                      emin_pattern_t** out) {
  if (!out) return EMIN_ERR_ARG;
  *out = nullptr;
  emin_pattern_t* h = nullptr;
  emin_status st = guarded([&] {
    check_system(sys);
    check_params(prm);
    if (ncp < 0 || (ncp && !cp)) throw Error(EMIN_ERR_ARG, "C point list");
    if (ncp > sys->Bdiv.nrows) throw Error(EMIN_ERR_SHAPE, "more C points than pressures");
    h = new emin_pattern_s();
    build_pattern(h, sys, prm, as_stream(stream), cp, ncp);
  });
  if (st != EMIN_OK) {
    if (h) {
      (void)hipStreamSynchronize(as_stream(stream));
      delete h;
    }
    return st;
  }
  set_last_error("");
  *out = h;
  return EMIN_OK;
}

emin_status emin_setup_with_pattern_noalloc(const emin_csr_t* M, const int64_t* N_rowptr,
                                            const int32_t* N_col, int64_t ncoarse, int64_t nnz_N,
                                            const int32_t* cid, const double* W, const double* Wc,
                                            int32_t iters, int32_t precision, uint32_t flags,
                                            double* P_vals, void* stream, emin_report_t* report) {
  return guarded([&] {
    if (!M) throw Error(EMIN_ERR_ARG, "NULL operator");
    if (M->nrows < 0 || M->nnz < 0 || ncoarse < 0 || nnz_N < 0)
      throw Error(EMIN_ERR_ARG, "negative size");
    if (flags & EMIN_FLAG_STAGED_PRODUCT)
      throw Error(EMIN_ERR_ARG, "the staged product is not available without allocation");
    // the pattern's longest row is not known before it is read; the bound
    // takes the largest map (4 planes)
    const size_t need = setup_with_pattern_bytes(M->nrows, ncoarse, nnz_N, M->nnz, 64);
    if (need > kScratchBytes)
      throw Error(EMIN_ERR_CAPACITY, "problem larger than the 64 MiB scratch buffer");
    Arena ar(scratch_ptr(), kScratchBytes);
    try {
      run_setup_with_pattern(M, N_rowptr, N_col, ncoarse, nnz_N, cid, W, Wc, iters, precision,
                             flags, P_vals, as_stream(stream), report, &ar);
    } catch (...) {
      (void)hipStreamSynchronize(as_stream(stream));
      throw;
    }
  });
}

emin_status emin_setup_with_pattern(const emin_csr_t* M, const int64_t* N_rowptr,
                                    const int32_t* N_col, int64_t ncoarse, int64_t nnz_N,
                                    const int32_t* cid, const double* W, const double* Wc,
                                    int32_t iters, int32_t precision, uint32_t flags,
                                    double* P_vals, void* stream, emin_report_t* report) {
  return guarded([&] {
    try {
      run_setup_with_pattern(M, N_rowptr, N_col, ncoarse, nnz_N, cid, W, Wc, iters, precision,
                             flags, P_vals, as_stream(stream), report);
    } catch (...) {
      // the call's workspace is gone: let no queued kernel outlive it
      (void)hipStreamSynchronize(as_stream(stream));
      throw;
    }
  });
}

emin_status emin_autotune_stats(int64_t* out4) {
  if (!out4) return EMIN_ERR_ARG;
  emin::autotune_stats(out4);
  return EMIN_OK;
}

emin_status emin_autotune_reset(void) {
  emin::autotune_clear();
  return EMIN_OK;
}

emin_status emin_pattern_info(const emin_pattern_t* h, emin_sizes_t* out) {
  if (!h || !out) return EMIN_ERR_ARG;
  *out = h->sizes;
  // the handle keeps allocating after the pattern phase (FP32 RAP copies,
  // GMRES workspace): report what it holds now
  out->device_bytes = (int64_t)h->ar.bytes();
  return EMIN_OK;
}

emin_status emin_pattern_view(const emin_pattern_t* h, int32_t what, emin_view_t* out) {
  if (!h || !out) return EMIN_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  auto csr = [&](const Csr& c, bool with_val) {
    out->n = c.nrows;
    out->ncols = c.ncols;
    out->nnz = c.nnz;
    out->rowptr = c.rowptr;
    out->col = c.col;
    out->val = with_val ? c.val : nullptr;
  };
  auto arr = [&](int64_t n, const void* p) {
    out->n = n;
    out->data = p;
  };
  switch (what) {
    case EMIN_VIEW_PV: csr(h->vp.N, false); break;
    case EMIN_VIEW_PP: csr(h->cp.N, false); break;
    case EMIN_VIEW_AC: csr(h->Ac, false); break;
    case EMIN_VIEW_BC: csr(h->Bc, false); break;
    case EMIN_VIEW_MV: csr(energy_v(h), true); break;
    case EMIN_VIEW_MP: csr(h->Mp, true); break;
    case EMIN_VIEW_S: csr(h->cp.S, false); break;
    case EMIN_VIEW_ORDER: arr(h->cp.n_c, h->ca.order); break;
    case EMIN_VIEW_CP: arr(h->cp.n_c, h->cp.clist); break;
    case EMIN_VIEW_CBAR: arr(h->n_p, h->cbar); break;
    case EMIN_VIEW_CV: arr(h->vp.n_c, h->vp.clist); break;
    case EMIN_VIEW_XVC: arr(h->vp.n_c * h->dim, h->xv_c); break;
    case EMIN_VIEW_P2VC: arr(h->cp.n_c, h->p2v_c); break;
    case EMIN_VIEW_KEEPV: arr(h->nnzA, h->keep_v); break;
    case EMIN_VIEW_KEEPP: arr(h->Z.nnz, h->keep_p); break;
    case EMIN_VIEW_DIR: arr(h->n_v, h->dir); break;
    default: return EMIN_ERR_ARG;
  }
  return EMIN_OK;
}

emin_status emin_setup(emin_pattern_t* h, const emin_system_t* sys, const emin_params_t* prm,
                       double* Pv_vals, double* Pp_vals, void* stream, emin_report_t* report) {
  if (!h) return EMIN_ERR_ARG;
  return guarded([&] { run_setup(h, sys, prm, Pv_vals, Pp_vals, as_stream(stream), report); });
}

emin_status emin_setup_pg(emin_pattern_t* h, const emin_system_t* sys, const emin_params_t* prm,
                          double* Pv_vals, double* Pp_vals, double* Rvt_vals, void* stream,
                          emin_report_t* report) {
  if (!h) return EMIN_ERR_ARG;
  return guarded([&] {
    if (!h->pg) throw Error(EMIN_ERR_ARG, "pattern built without EMIN_FLAG_PETROV_GALERKIN");
    if (h->sizes.nnz_Pv && !Rvt_vals) throw Error(EMIN_ERR_ARG, "NULL Rvt");
    run_setup(h, sys, prm, Pv_vals, Pp_vals, as_stream(stream), report,
              Rvt_vals ? Rvt_vals : reinterpret_cast<double*>(h->ar.alloc<double>(1)));
  });
}

emin_status emin_rap_pg(emin_pattern_t* h, const emin_system_t* sys, const double* Pv_vals,
                        const double* Pp_vals, const double* Rvt_vals, double* Ac_vals,
                        double* Bc_vals, double* Gct_vals, void* stream) {
  if (!h) return EMIN_ERR_ARG;
  return guarded([&] {
    run_rap_pg(h, sys, Pv_vals, Pp_vals, Rvt_vals, Ac_vals, Bc_vals, Gct_vals, as_stream(stream));
  });
}

emin_status emin_rap(emin_pattern_t* h, const emin_system_t* sys, const double* Pv_vals,
                     const double* Pp_vals, double* Ac_vals, double* Bc_vals, int32_t precision,
                     void* stream) {
  if (!h) return EMIN_ERR_ARG;
  return guarded([&] {
    run_rap(h, sys, Pv_vals, Pp_vals, Ac_vals, Bc_vals, precision, as_stream(stream));
  });
}

emin_status emin_sync_report(const emin_report_t* report, void* stream, emin_report_t* host) {
  if (!report || !host) return EMIN_ERR_ARG;
  return guarded([&] {
    HIP_OK(hipMemcpyAsync(host, report, sizeof(emin_report_t), hipMemcpyDeviceToHost,
                          as_stream(stream)));
    HIP_OK(hipStreamSynchronize(as_stream(stream)));
    if (host->status != EMIN_OK) throw Error((emin_status)host->status, "numeric phase");
  });
}

emin_status emin_memcpy_d2h(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return EMIN_OK;
  if (!dst || !src) return EMIN_ERR_ARG;
  return guarded([&] {
    HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, as_stream(stream)));
    HIP_OK(hipStreamSynchronize(as_stream(stream)));
  });
}

void emin_pattern_destroy(emin_pattern_t* h) {
  if (!h) return;
  delete h;
}

const char* emin_status_string(emin_status s) {
  switch (s) {
    case EMIN_OK: return "OK";
    case EMIN_ERR_ARG: return "ERR_ARG";
    case EMIN_ERR_SHAPE: return "ERR_SHAPE";
    case EMIN_ERR_PATTERN: return "ERR_PATTERN";
    case EMIN_ERR_VALUE: return "ERR_VALUE";
    case EMIN_ERR_INFEASIBLE: return "ERR_INFEASIBLE";
    case EMIN_ERR_BREAKDOWN: return "ERR_BREAKDOWN";
    case EMIN_ERR_BUDGET: return "ERR_BUDGET";
    case EMIN_ERR_DEVICE: return "ERR_DEVICE";
    case EMIN_ERR_OOM: return "ERR_OOM";
    case EMIN_ERR_CAPACITY: return "ERR_CAPACITY";
    case EMIN_ERR_COLOCATE: return "ERR_COLOCATE";
    case EMIN_ERR_CANCELLED: return "ERR_CANCELLED";
  }
  return "UNKNOWN";
}

const char* emin_version(void) { return "emin-mi355x 0.1.0 (gfx950)"; }

const char* emin_last_error(void) { return g_last_error.c_str(); }

emin_status emin_fp_probe(const double* x, double* out_sqrt, double* out_rcp, int64_t n,
                          void* stream) {
  if (n < 0 || (n && (!x || !out_sqrt || !out_rcp))) return EMIN_ERR_ARG;
  return guarded([&] {
    if (n) k_fp_probe<<<nblocks(n, 256), 256, 0, as_stream(stream)>>>(x, out_sqrt, out_rcp, n);
    HIP_OK(hipGetLastError());
  });
}

}  // extern "C"
