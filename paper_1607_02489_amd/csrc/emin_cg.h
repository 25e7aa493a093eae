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
  int32_t unroll = 4;              // map rows: M entries whose gathers are issued together
};

// options of a masked-product schedule (the autotuner's search space)
struct SchedOpts {
  bool maps = true;      // rows that fit the intersection maps use them
  int gshift = 0;        // lanes per row: the tight power of two, times 2^gshift
  int xcd_split = XCD_MERGED;   // XCD_*
  bool stage = false;    // blocks of rows whose Z rows fit in LDS use the staged kernel
  int unroll = 4;        // map rows: gathers in flight per lane (4 or 16)
};

// sizes of the LDS-staged masked product: sr rows per block, at most emax M
// entries, vcap staged Z values and rcap runs of consecutive Z rows; np map
// planes
struct StageDims {
  int32_t sr = 16, emax = 640, rcap = 64, vcap = 3072, np = 1;
};

// plan of the staged product (built once per pattern): the staged blocks of
// sr rows, per block its runs of Z rows (start in Z, start in LDS, length) and
// per M entry the LDS position its intersection map is relative to
struct StagePlan {
  StageDims dims;
  int64_t nblk = 0;                 // staged blocks
  const int32_t* blocks = nullptr;  // their indices (block b: rows [b sr, b sr + sr))
  const int64_t* roff = nullptr;    // per block of the matrix: its first run (nb + 1)
  const int32_t *rg = nullptr, *rl = nullptr, *rn = nullptr;
  const int32_t* lofs = nullptr;    // per M entry of a staged row
  const uint8_t* row_staged = nullptr;
  int64_t rows = 0, m_entries = 0, p_entries = 0;   // covered by staged blocks
};

// kernel arguments of the staged product
struct StageArgs {
  StageDims dims;
  const int32_t* blocks;
  const int64_t* roff;
  const int32_t *rg, *rl, *rn;
  const int32_t* lofs;
  int64_t n;
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
  StagePlan stage;
  // stage: blocks whose Z rows fit in LDS use the staged kernel
  void make_bins(const Csr& M, const int64_t* nrp, const int32_t* ncol, hipStream_t s, Arena& ar,
                 bool tune, bool stage = false);
  int32_t sched_code() const;   // bit 0 maps, bit 1 doubled lanes, bit 2 XCD split, bits 4-5
                                // tuned, bit 6 staged blocks, bit 7 4-entry gather batches
};

// the staged product's plan (rows in blocks that fit LDS), and the product on
// those blocks (spmm_stage.hip)
void stage_plan(EminWork& w, const Csr& M, const int64_t* nrp, const uint8_t* elig, hipStream_t s,
                Arena& ar);
template <class TM, class TX, class TY>
void spmm_stage(const EminWork& w, const int64_t* mrp, const TM* mval, const int64_t* nrp,
                const TX* X, TY* Y, const double* Dv, double bytes, hipStream_t s);

// Y = mask_N(M X).  With D, also <D, Y>: *dots receives the array of values
// whose in-order sum is that scalar and the return value is their count.
int64_t masked_spmm(const EminWork& w, const Csr& M, const int64_t* nrp, const int32_t* ncol,
                    const double* X, double* Y, const double* D, double* part,
                    const double** dots, hipStream_t s);

void run_emin(EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp, const int32_t* ncol,
              const int32_t* cid, const int32_t* clist, const double* W, double* P, int iters,
              bool energy, bool mixed, EminReportPtrs rp, hipStream_t s);

// Krylov workspace of the GMRES form (emin_gmres.hip), grown on demand
struct GmresWork {
  int cap = -1;
  double *V = nullptr, *H = nullptr, *y = nullptr, *state = nullptr;
  void reserve(int iters, int64_t nnz, int64_t np, Arena& ar);
};

// sec. 4.3 in its GMRES form for a non-symmetric operator M: `iters` steps
// of GMRES on Pi mask_N(M P) = 0 from P0; the report's rho holds the squared
// residual norms
void run_emin_gmres(EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp,
                    const int32_t* ncol, const int32_t* cid, const int32_t* clist, const double* W,
                    double* P, int iters, bool mixed, EminReportPtrs rp, GmresWork& gw,
                    hipStream_t s);

// building blocks shared by the CG and GMRES forms
void gather_modes(const double* W, const int32_t* clist, int64_t nc, double* Wc, hipStream_t s);
void emin_init(const int64_t* rp, const int32_t* col, int64_t n, const int32_t* cid,
               const double* W, const double* Wc, double* G, double* P, int32_t* status,
               hipStream_t s);
// Y = mask_N(M X) in FP64, or from FP32 copies (M's in Mf, X's made here)
void masked_product(const EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp,
                    const int32_t* ncol, const double* X, double* Y, bool mixed, hipStream_t s);

void default_modes(const uint8_t* dir, int64_t n, double* W, hipStream_t s);
// autotuner bookkeeping: timed shapes, reuses, candidates timed, table size
void autotune_stats(int64_t* out);
void autotune_clear();
void to_float(const double* a, float* b, int64_t n, hipStream_t s);

}  // namespace emin
