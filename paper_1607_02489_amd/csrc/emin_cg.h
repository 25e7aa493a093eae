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
// threads per block of the masked product (a multiple of 64)
constexpr int SPMM_BS = 64;

// block order of the masked product over the XCDs
enum : int32_t {
  XCD_CONTIGUOUS = 0,   // each XCD takes one contiguous eighth of the grid
  XCD_BY_CLASS = 1,     // each XCD takes an eighth of every row class
  XCD_MERGED = 2        // blocks of all classes in order of their first row, then
                        // one contiguous eighth of that order per XCD
};

struct SpmmSched {
  const int32_t* rows = nullptr;
  int64_t row_off[SPMM_NT + 1] = {};
  int64_t blk_off[SPMM_NT + 1] = {};
  int32_t xcd_split = XCD_BY_CLASS;
  const int32_t* bmap = nullptr;   // XCD_MERGED: (class << 27) | block in class, per slot
};

// options of a masked-product schedule (the autotuner's search space)
struct SchedOpts {
  bool maps = true;      // rows that fit the intersection maps use them
  int gshift = 0;        // lanes per row: the tight power of two, times 2^gshift
  int xcd_split = XCD_MERGED;   // XCD_*
};

struct EminWork {
  int64_t n = 0, nnz = 0, nc = 0;
  int g = 8;       // lanes per row of the masked product
  int smax = 8;    // longest pattern row
  double *G = nullptr, *Wc = nullptr, *Wdef = nullptr;
  double *R = nullptr, *Z = nullptr, *Q = nullptr, *MP = nullptr;
  float *Zf = nullptr, *Qf = nullptr;
  double *part = nullptr, *part_e = nullptr;
  double* rowdot = nullptr;   // per-row <D, Y> of the last masked product (0 for empty rows)
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
  int tuned = 0;   // 0: default schedule, 1: timed here, 2: reused from the tuning table
  SchedOpts opts;
  void make_bins(const Csr& M, const int64_t* nrp, const int32_t* ncol, hipStream_t s, Arena& ar,
                 bool tune);
  int32_t sched_code() const;   // bit 0 maps, bit 1 doubled lanes, bit 2 XCD split, bits 4-5 tuned
};

// Y = mask_N(M X).  With D, also <D, Y>: *dots receives the array of values
// whose in-order sum is that scalar and the return value is their count.
int64_t masked_spmm(const EminWork& w, const Csr& M, const int64_t* nrp, const int32_t* ncol,
                    const double* X, double* Y, const double* D, double* part,
                    const double** dots, hipStream_t s);

void run_emin(EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp, const int32_t* ncol,
              const int32_t* cid, const int32_t* clist, const double* W, double* P, int iters,
              bool energy, bool mixed, EminReportPtrs rp, hipStream_t s);

void default_modes(const uint8_t* dir, int64_t n, double* W, hipStream_t s);
// autotuner bookkeeping: timed shapes, reuses, candidates timed, table size
void autotune_stats(int64_t* out);
void autotune_clear();
void to_float(const double* a, float* b, int64_t n, hipStream_t s);

}  // namespace emin
