// Coarse-point selection and sparsity patterns (Alg. 3, Alg. 4, sec. 4.2).
#pragma once
#include <functional>

#include "common.h"

namespace emin {

enum : uint8_t { ST_U = 0, ST_CAND = 1, ST_F = 2, ST_C = 3 };

// state of Alg. 3 on one graph (passed by value to the kernels)
struct CoarsenArgs {
  const int64_t* grp = nullptr;   // graph: structure of the filtered operator
  const int32_t* gcol = nullptr;
  int64_t n = 0;
  int dim = 2;
  const double* x = nullptr;      // n*dim coordinates
  uint8_t* st = nullptr;          // ST_*
  int32_t* cnt = nullptr;         // C points within distance 4
  double* rs = nullptr;           // sum of 1/|x_j - x_c| over those C points
  double* hkey = nullptr;         // h1 = cnt/rs of a candidate, +inf otherwise
  int32_t* s_cnt = nullptr;       // |S_j|
  int32_t* s_c = nullptr;         // S_j entries (n*scap), insertion order until sorted
  uint8_t* s_d = nullptr;         // their graph distances
  int scap = 32;
  int32_t* order = nullptr;       // C points in selection order
  int32_t* meta = nullptr;        // [0] |C|, [1] |C| of Alg. 3, [2] error bits
  const int32_t* balls = nullptr; // distance-4 balls (vertex | dist << 29), n*bmax
  const int32_t* bsize = nullptr; // ball sizes
  const int32_t* b3 = nullptr;    // entries at distance <= 3 (a prefix of the ball)
  int bmax = 0;                   // largest ball
  int64_t bstride = 0;            // row stride of balls (>= bmax)
  int vb = 64;                    // vertices per argmin block
  int nblk = 1;
  int dcap = 1024;
};

struct CoarsenOut {
  int64_t n_c = 0, n_alg3 = 0;
  int32_t* cid = nullptr;    // coarse index of a C point, -1 for F
  int32_t* clist = nullptr;  // C points, ascending
  Csr N;                     // N^(p) pattern (val unused)
  Csr S;                     // S sets (fine indices, sorted)
  uint8_t* sdist = nullptr;
};

// Alg. 3 and the extra distance-3 points, or, with cp_given (ncp ascending
// fine indices, device memory), that C^(p) taken as given.  overlap, when
// given, is called once the single-workgroup kernels are queued and before
// the host waits for them, so that independent work the caller queues on
// another stream runs beside them.
void coarsen_pressure(CoarsenArgs& D, CoarsenOut& out, hipStream_t s, Arena& ar, int lds_max,
                      const int32_t* cp_given = nullptr, int64_t ncp = 0,
                      const std::function<void()>& overlap = nullptr);

// Alg. 4: C-bar^(p) flags (n_p) from the S sets; returns |C-bar^(p)| (the C
// points and the mid-points added)
int64_t midpoints(const Csr& S, const uint8_t* st, const double* x, int dim, double tau2_sq,
                  uint8_t* cbar, hipStream_t s, Arena& ar, int lds_max);

// sec. 4.2: C^(v) (flags in/out, n_v) with the extra points and the N^(v)
// pattern (coarse columns); returns the number of extra points
struct VPatternOut {
  Csr N;
  int32_t* cid = nullptr;
  int32_t* clist = nullptr;
  int64_t n_c = 0, n_extra = 0;
};
void velocity_pattern(const Csr& G, const uint8_t* dir, uint8_t* cv, VPatternOut& out,
                      hipStream_t s, Arena& ar, int lds_max);

}  // namespace emin
