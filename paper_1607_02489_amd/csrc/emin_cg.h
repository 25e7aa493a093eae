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

struct EminWork {
  int64_t n = 0, nnz = 0, nc = 0;
  int g = 8;       // lanes per row of the masked product
  int smax = 8;    // longest pattern row
  double *G = nullptr, *Wc = nullptr, *Wdef = nullptr;
  double *R = nullptr, *Z = nullptr, *Q = nullptr, *MP = nullptr;
  float *Zf = nullptr, *Qf = nullptr;
  double *part = nullptr, *part_e = nullptr;
  CgScalars* sc = nullptr;
  // row bins of the masked product by pattern-row length: (0,4], (4,8], ..., (32,64];
  // mbin_*: rows served from precomputed intersection maps (length <= 32),
  // bin_*: the rest, served by the searching kernel
  static constexpr int NBIN = 5;
  int32_t* bin_rows[NBIN] = {};
  int64_t bin_n[NBIN] = {};
  int32_t* mbin_rows[NBIN] = {};
  int64_t mbin_n[NBIN] = {};
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
