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
  bool stage = false;    // rows of tiles whose Z rows fit in LDS use the tiled kernel
  int unroll = 4;        // map rows: gathers in flight per lane (4 or 16)
};

// sizes of the tiled masked product: rows are grouped by the cells of a
// grid over their coordinates (about tgt rows per cell); a cell of at most
// tmax rows is staged when its union of Z rows spans a k window of at most
// wbits, holds at most vcap values and forms at most rcap runs
struct TileDims {
  int32_t tgt = 64, tmax = 256, vcap = 4096, rcap = 128, wbits = 131072;
};

// waves of a tile workgroup
constexpr int TILE_WAVES = 8;

// plan of the tiled product (built once per pattern): per staged tile its
// record (first row in srows, rows per slots class (<= 8, <= 16), unused,
// first run, runs, staged values, cell), the staged rows tile by tile with
// each one's first M entry, M length, first pattern entry and slots (smeta),
// the runs of consecutive Z rows (start in Z, start in LDS, length) and per M
// entry of a staged row the LDS position its intersection map is relative to
struct StagePlan {
  TileDims dims;
  int64_t ntile = 0;
  const int32_t* tinfo = nullptr;
  const int32_t* srows = nullptr;
  const int4* smeta = nullptr;
  const int32_t *rg = nullptr, *rl = nullptr, *rn = nullptr;
  const int32_t* lofs = nullptr;
  const uint8_t* row_staged = nullptr;
  int32_t vmax = 0;                                // largest tile's staged values
  int64_t rows = 0, m_entries = 0, p_entries = 0;  // covered by staged tiles
};

// kernel arguments of the tiled product
struct StageArgs {
  const int32_t* tinfo;
  const int32_t* srows;
  const int4* smeta;
  const int32_t *rg, *rl, *rn;
  const int32_t* lofs;
  int32_t zbytes;   // LDS bytes of the staged Z values (16-byte aligned)
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
  // (nplanes words of eight fields, plane-major, planes nnzm apart)
  int32_t* kofs = nullptr;
  uint32_t* nib = nullptr;
  int64_t nnzm = 0;
  int nplanes = 1;
  void allocate(int64_t n, int64_t nnz, int64_t nc, Arena& ar, bool mixed);
  int tuned = 0;   // 0: default schedule, 1: timed here, 2: reused from the tuning table
  SchedOpts opts;
  StagePlan stage;
  // stage: rows in tiles whose Z rows fit in LDS use the tiled kernel; the
  // tiles come from the rows' coordinates (row i at xyz[(xmap ? xmap[i] :
  // i) * dim ...]), or from blocks of consecutive rows without them
  void make_bins(const Csr& M, const int64_t* nrp, const int32_t* ncol, hipStream_t s, Arena& ar,
                 bool tune, bool stage = false, const double* xyz = nullptr,
                 const int32_t* xmap = nullptr, int dim = 0);
  int32_t sched_code() const;   // bit 0 maps, bit 1 doubled lanes, bit 2 XCD split, bits 4-5
                                // tuned, bit 6 tiled rows, bit 7 16-entry gather batches
};

// the tiled product's plan, and the product on the staged tiles
// (spmm_stage.hip); e0 / e1, when given, are recorded at the launch's start
// and end
void stage_plan(EminWork& w, const Csr& M, const int64_t* nrp, const uint8_t* elig,
                const double* xyz, const int32_t* xmap, int dim, hipStream_t s, Arena& ar);
template <class TM, class TX, class TY>
void spmm_stage(const EminWork& w, const int64_t* mrp, const TM* mval, const int64_t* nrp,
                const TX* X, TY* Y, const double* Dv, hipStream_t s, hipEvent_t e0,
                hipEvent_t e1);

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
void emin_init(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz,
               const int32_t* cid,
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
