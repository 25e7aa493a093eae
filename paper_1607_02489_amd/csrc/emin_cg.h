// EMIN-AMG constrained CG (sec. 4.3) on one block (scalar velocity or pressure).
#pragma once
#include "common.h"

namespace emin {

struct CgScalars {
  double rho, alpha, beta;
  int32_t stop, its;
};

struct EminReportPtrs {
  double* energy = nullptr;   // iters+1
  double* rho = nullptr;      // iters+1
  double* gamma = nullptr;    // iters
  int32_t* its = nullptr;
  int32_t* status = nullptr;
};

// one masked-product launch: row lists of every class back to back, with the
// row and block ranges of each class
constexpr int SPMM_NT = 9;
struct SpmmSched {
  const int32_t* rows = nullptr;
  int64_t row_off[SPMM_NT + 1] = {};
  int64_t blk_off[SPMM_NT + 1] = {};
};

struct EminWork {
  int64_t n = 0, nnz = 0, nc = 0;
  int g = 8;       // lanes per row of the masked product
  int smax = 8;    // longest pattern row
  double *G = nullptr, *Wc = nullptr, *Wdef = nullptr;
  double *R = nullptr, *Z = nullptr, *Q = nullptr, *MP = nullptr;
  float *Zf = nullptr, *Qf = nullptr;
  double *part = nullptr, *part_e = nullptr;
  CgScalars* sc = nullptr;
  // row classes of the masked product by pattern-row length: rows served
  // from precomputed intersection maps (length <= 32, G = 4..32) and the rest,
  // served by the searching kernel (G = 4..64)
  SpmmSched sched;
  // intersection maps per M entry: base offset and 4-bit slot fields
  // (nplanes words of eight fields, plane-major)
  int32_t* kofs = nullptr;
  uint32_t* nib = nullptr;
  int64_t nnzm = 0;
  int nplanes = 1;
  void allocate(int64_t n, int64_t nnz, int64_t nc, Arena& ar, bool mixed);
  void make_bins(const Csr& M, const int64_t* nrp, const int32_t* ncol, hipStream_t s, Arena& ar);
};

// Y = mask_N(M X) with <D, Y> block partials (D may be NULL); returns the
// number of partials written
int64_t masked_spmm(const EminWork& w, const Csr& M, const int64_t* nrp, const int32_t* ncol,
                    const double* X, double* Y, const double* D, double* part, hipStream_t s);

void run_emin(EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp, const int32_t* ncol,
              const int32_t* cid, const int32_t* clist, const double* W, double* P, int iters,
              bool energy, bool mixed, EminReportPtrs rp, hipStream_t s);

void default_modes(const uint8_t* dir, int64_t n, double* W, hipStream_t s);
void to_float(const double* a, float* b, int64_t n, hipStream_t s);

}  // namespace emin
