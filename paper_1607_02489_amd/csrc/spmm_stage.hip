// Masked product Q = mask_N(M Z) on spatial tiles with LDS-staged rows of Z
// (sec. 4.3).
//
// The rows are grouped into tiles by the cells of a uniform grid laid over
// their coordinates (cells sized for about 64 rows).  A tile's rows reach a
// set of Z rows k (the union of their M rows' columns) several times smaller
// than the sum of their lengths: neighbouring mesh nodes share most of their
// neighbours.  A workgroup copies that union into LDS once, as runs of
// consecutive k (pattern rows are stored back to back, so a run of k's is one
// contiguous stretch of Z's values: a coalesced stream), and every gather of
// the product then reads LDS.  L2 and HBM see each Z row once per tile
// instead of once per (i, k) pair.
//
// Within a tile the rows are processed in packs of eight rows by one wave,
// eight lanes per row: lane l takes the row's M entries l, l + 8, l + 16, ...
// (coalesced loads straight into registers, the next eight loaded while the
// current eight are summed) and keeps one partial sum per slot of the row
// (rows of at most 16 slots; longer ones keep the gathering kernel).  A
// slot's eight partials are then added in a fixed tree on the DPP network.
// The order is fixed, so results are deterministic; it differs from the
// gathering kernel's ascending-k sum only by rounding.  The plan (tiles,
// their runs, each M entry's LDS offset) is built once per pattern.
#include "emin_cg.h"
#include "prof.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace emin {

namespace {

constexpr int PL_BS = 256;   // threads of a plan block (one cell)
constexpr int TINFO = 8;     // ints of a tile's record

// ---------------------------------------------------------------------------
// cells
// ---------------------------------------------------------------------------
struct CellGrid {
  double lo[3];
  double inv;      // 1 / cell size
  int32_t nc[3];   // cells per dimension
  int32_t ncell;
};

__device__ __forceinline__ double coord(const double* xyz, const int32_t* xmap, int dim,
                                        int64_t i, int d) {
  const int64_t v = xmap ? (int64_t)xmap[i] : i;
  return xyz[v * dim + d];
}

// Bounding box of the rows' coordinates and the cell size that gives about
// tgt rows per cell over the box (a dimension of zero extent takes one
// cell); the cell grows until the cell count is within cap.  One block.
__global__ __launch_bounds__(1024) void k_cell_grid(const double* xyz, const int32_t* xmap,
                                                    int dim, int64_t n, int tgt, int64_t cap,
                                                    CellGrid* g) {
  __shared__ double smin[3][16], smax[3][16];
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    for (int d = 0; d < dim; d++) {
      const double v = coord(xyz, xmap, dim, i, d);
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
    }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 0; d < 3; d++) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      mn[d] = fmin(mn[d], __shfl_xor(mn[d], m, 64));
      mx[d] = fmax(mx[d], __shfl_xor(mx[d], m, 64));
    }
    if (lane == 0) {
      smin[d][w] = mn[d];
      smax[d][w] = mx[d];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double lo[3], ext[3];
  for (int d = 0; d < 3; d++) {
    double a = 1e300, b = -1e300;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) {
      a = fmin(a, smin[d][k]);
      b = fmax(b, smax[d][k]);
    }
    lo[d] = d < dim ? a : 0.0;
    ext[d] = d < dim && b > a ? b - a : 0.0;
  }
  double vol = 1.0;
  int de = 0;
  for (int d = 0; d < dim; d++)
    if (ext[d] > 0.0) {
      vol *= ext[d];
      de++;
    }
  double cs = de ? pow(vol * (double)tgt / (double)(n > 0 ? n : 1), 1.0 / de) : 1.0;
  if (!(cs > 0.0)) cs = 1.0;
  int32_t nc[3] = {1, 1, 1};
  for (int it = 0; it < 400; it++) {
    double tot = 1.0;
    for (int d = 0; d < 3; d++) {
      nc[d] = ext[d] > 0.0 ? (int32_t)fmin(floor(ext[d] / cs) + 1.0, 1e9) : 1;
      tot *= (double)nc[d];
    }
    if (tot <= (double)cap) break;
    cs *= 1.25;
  }
  for (int d = 0; d < 3; d++) {
    g->lo[d] = lo[d];
    g->nc[d] = nc[d];
  }
  g->inv = 1.0 / cs;
  g->ncell = nc[0] * nc[1] * nc[2];
}

// each row's cell (z-major, then y, then x), counted per cell (cnt[c + 1]);
// without coordinates, blocks of tgt consecutive rows
__global__ void k_cell_key(const double* xyz, const int32_t* xmap, int dim, int64_t n, int tgt,
                           const CellGrid* g, int32_t* key, int64_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c;
  if (xyz) {
    int32_t q[3] = {0, 0, 0};
    for (int d = 0; d < dim; d++) {
      const double t = (coord(xyz, xmap, dim, i, d) - g->lo[d]) * g->inv;
      q[d] = (int32_t)fmax(0.0, fmin(floor(t), (double)(g->nc[d] - 1)));
    }
    c = (q[2] * g->nc[1] + q[1]) * g->nc[0] + q[0];
  } else {
    c = (int32_t)(i / tgt);
  }
  key[i] = c;
  atomicAdd(reinterpret_cast<unsigned long long*>(cnt + c + 1), 1ull);
}

// rows placed by cell (the order within a cell is settled by the plan)
__global__ void k_cell_place(const int32_t* key, int64_t n, const int64_t* coff, int32_t* cur,
                             int32_t* csort) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t c = key[i];
  csort[coff[c] + atomicAdd(&cur[c], 1)] = (int32_t)i;
}

__device__ __forceinline__ int block_excl_scan(int v, int* tmp) {
  // exclusive scan over the block (PL_BS threads); tmp holds PL_BS/64 + 1
  // ints, and its total stays in tmp[PL_BS/64] until the next call
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();   // every thread has read the previous call's tmp
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0;
    for (int k = 0; k < PL_BS / 64; k++) {
      const int t = tmp[k];
      tmp[k] = a;
      a += t;
    }
    tmp[PL_BS / 64] = a;
  }
  __syncthreads();
  return tmp[w] + x - v;
}

struct PlanArgs {
  TileDims D;
  const int64_t* mrp;
  const int32_t* mcol;
  const int64_t* nrp;
  const int32_t* kofs;
  const uint8_t* elig;
  const int64_t* coff;
  const int32_t* csort;
  // pass 0 outputs
  uint8_t* flag;
  int64_t* nrun;                // per cell: runs of a staged cell, else 0
  int32_t* vmax;
  unsigned long long* cnt;      // staged rows, their M entries, their pattern entries, tiles
  // pass 1
  const int64_t* tix;           // inclusive scan of the flags
  const int64_t* roff;          // inclusive scan of nrun
  int32_t* tinfo;
  int32_t* srows;
  int4* smeta;
  int32_t *rg, *rl, *rn;
  int32_t* lofs;
  uint8_t* row_staged;
};

// LDS of a plan block
__host__ __device__ constexpr size_t plan_lds(const TileDims& D) {
  return (size_t)D.tmax * (8 + 8 + 4 + 4)     // M starts, sort keys, rows, entry prefix
         + (size_t)(D.wbits >> 5) * 8          // bitmap words and their ranks
         + (size_t)(2 * D.vcap + 1) * 4;       // union entries and offsets
}

// Plan of one cell.  Its rows that fit the tiled kernel (map-eligible, 1 to
// 32 slots) are staged when the cell has at most tmax rows and the union of
// their Z rows fits (k window, values, runs).  Pass 0 decides and counts;
// pass 1 (staged cells) writes the runs, the LDS offset of every M entry of a
// staged row, the staged rows ordered by (slots class, M length descending,
// index) and the tile's record.  The M entries of the staged rows are walked
// as one flat range (each thread a stride of it), the row of an entry found
// by binary search over the rows' entry prefix.
template <int PASS>
__global__ __launch_bounds__(PL_BS) void k_tile_plan(PlanArgs A) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const TileDims& D = A.D;
  const int nw = D.wbits >> 5;
  int64_t* s_ma = reinterpret_cast<int64_t*>(dsm);                // rows' first M entry
  uint64_t* s_key = reinterpret_cast<uint64_t*>(s_ma + D.tmax);   // staged rows' sort keys
  uint32_t* bits = reinterpret_cast<uint32_t*>(s_key + D.tmax);
  int32_t* wpre = reinterpret_cast<int32_t*>(bits + nw);
  int32_t* s_u = wpre + nw;
  int32_t* s_off = s_u + D.vcap;
  int32_t* s_row = s_off + D.vcap + 1;   // rows of the cell (-1: not staged)
  int32_t* s_pre = s_row + D.tmax;       // exclusive prefix of staged rows' M lengths
  __shared__ int tmp[PL_BS / 64 + 1];
  __shared__ int s_kmin, s_kmax;
  const int64_t c = blockIdx.x;
  if (PASS == 1 && !A.flag[c]) return;
  const int64_t r0 = A.coff[c], r1 = A.coff[c + 1];
  const int T = (int)(r1 - r0);
  const bool fits = T > 0 && T <= D.tmax;
  if (!fits) {
    if (PASS == 0 && threadIdx.x == 0) {
      A.flag[c] = 0;
      A.nrun[c] = 0;
    }
    return;
  }
  // (every later rejection is taken by all threads together, after a
  // barrier, from values every thread reads the same)
  auto reject = [&]() {
    if (PASS == 0 && threadIdx.x == 0) {
      A.flag[c] = 0;
      A.nrun[c] = 0;
    }
  };
  if (threadIdx.x == 0) {
    s_kmin = INT32_MAX;
    s_kmax = -1;
  }
  int mlen = 0;
  const int t = threadIdx.x;   // T <= tmax <= PL_BS: one row per thread
  if (t < T) {
    const int32_t i = A.csort[r0 + t];
    const int64_t ni = A.nrp[i + 1] - A.nrp[i];
    const bool ok = A.elig[i] && ni >= 1 && ni <= 16;
    s_row[t] = ok ? i : -1;
    s_ma[t] = A.mrp[i];
    mlen = ok ? (int)(A.mrp[i + 1] - A.mrp[i]) : 0;
    if (ok) {
      const uint64_t cl = ni <= 8 ? 0 : (ni <= 16 ? 1 : 2);
      const uint64_t ml = (uint64_t)(mlen < 0xFFFFF ? mlen : 0xFFFFF);
      s_key[t] = (cl << 60) | ((0xFFFFFull - ml) << 32) | (uint64_t)(uint32_t)i;
    }
  }
  const int pre = block_excl_scan(mlen, tmp);
  const int E = tmp[PL_BS / 64];   // M entries of the staged rows
  if (t < T) s_pre[t] = pre;
  __syncthreads();
  // row (local) of flat entry f: the last row whose prefix is <= f, among
  // rows with entries
  auto row_of = [&](int f) {
    int lo = 0, hi = T - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  if (E == 0) {
    reject();
    return;
  }
  // k window over the entries whose pattern row is not empty
  int kmn = INT32_MAX, kmx = -1;
  for (int f = t; f < E; f += PL_BS) {
    const int r = row_of(f);
    const int32_t k = A.mcol[s_ma[r] + (f - s_pre[r])];
    if (A.nrp[k + 1] == A.nrp[k]) continue;
    kmn = k < kmn ? k : kmn;
    kmx = k > kmx ? k : kmx;
  }
  if (kmx >= 0) {
    atomicMin(&s_kmin, kmn);
    atomicMax(&s_kmax, kmx);
  }
  __syncthreads();
  const int kmin = s_kmin, kmax = s_kmax;
  const int64_t width = kmax >= kmin ? (int64_t)kmax - kmin + 1 : 0;
  if (width == 0 || width > D.wbits) {
    reject();
    return;
  }
  const int nwu = (int)((width + 31) >> 5);
  for (int q = t; q < nwu; q += PL_BS) bits[q] = 0u;
  __syncthreads();
  for (int f = t; f < E; f += PL_BS) {
    const int r = row_of(f);
    const int32_t k = A.mcol[s_ma[r] + (f - s_pre[r])];
    if (A.nrp[k + 1] == A.nrp[k]) continue;
    const int o = k - kmin;
    atomicOr(&bits[o >> 5], 1u << (o & 31));
  }
  __syncthreads();
  // the union in ascending k: each thread a contiguous slice of words
  const int per = (nwu + PL_BS - 1) / PL_BS;
  const int w0 = t * per < nwu ? t * per : nwu;
  const int w1 = w0 + per < nwu ? w0 + per : nwu;
  int cu = 0;
  for (int q = w0; q < w1; q++) cu += __popc(bits[q]);
  int ub = block_excl_scan(cu, tmp);
  const int U = tmp[PL_BS / 64];
  if (U > D.vcap) {
    reject();
    return;
  }
  for (int q = w0; q < w1; q++) {
    wpre[q] = ub;
    uint32_t m = bits[q];
    while (m) {
      const int b = __ffs(m) - 1;
      m &= m - 1u;
      s_u[ub++] = kmin + 32 * q + b;
    }
  }
  __syncthreads();
  // staged values (pattern row lengths over the union) and runs
  const int pu = (U + PL_BS - 1) / PL_BS;
  const int u0 = t * pu < U ? t * pu : U;
  const int u1 = u0 + pu < U ? u0 + pu : U;
  int lv = 0, lr = 0;
  for (int u = u0; u < u1; u++) {
    const int32_t k = s_u[u];
    lv += (int)(A.nrp[k + 1] - A.nrp[k]);
    lr += (u == 0 || s_u[u - 1] != k - 1) ? 1 : 0;
  }
  int vb = block_excl_scan(lv, tmp);
  const int V = tmp[PL_BS / 64];
  int rb = block_excl_scan(lr, tmp);
  const int NR = tmp[PL_BS / 64];
  if (V > D.vcap || NR > D.rcap) {
    reject();
    return;
  }
  if (PASS == 0) {
    unsigned long long nr = 0, me = 0, pe = 0;
    if (t < T && s_row[t] >= 0) {
      nr = 1;
      me = (unsigned long long)mlen;
      pe = (unsigned long long)(A.nrp[s_row[t] + 1] - A.nrp[s_row[t]]);
    }
    if (nr) {
      atomicAdd(A.cnt + 0, nr);
      atomicAdd(A.cnt + 1, me);
      atomicAdd(A.cnt + 2, pe);
    }
    if (t == 0) {
      A.flag[c] = 1;
      A.nrun[c] = NR;
      atomicMax(A.vmax, V);
      atomicAdd(A.cnt + 3, 1ull);
    }
    return;
  }
  for (int u = u0; u < u1; u++) {
    s_off[u] = vb;
    vb += (int)(A.nrp[s_u[u] + 1] - A.nrp[s_u[u]]);
  }
  if (t == 0) s_off[U] = V;
  __syncthreads();
  const int64_t st = A.tix[c] - 1;
  const int64_t run0 = A.roff[c] - NR;
  for (int u = u0; u < u1; u++) {
    const int32_t k = s_u[u];
    if (u == 0 || s_u[u - 1] != k - 1) {
      int v = u + 1;
      while (v < U && s_u[v] == s_u[v - 1] + 1) v++;
      A.rg[run0 + rb] = (int32_t)A.nrp[k];
      A.rl[run0 + rb] = s_off[u];
      A.rn[run0 + rb] = s_off[v] - s_off[u];
      rb++;
    }
  }
  // every M entry of a staged row: its Z row's LDS start plus the map's base
  // shift (an entry whose pattern row is empty never matches: offset 0)
  for (int f = t; f < E; f += PL_BS) {
    const int r = row_of(f);
    const int64_t e = s_ma[r] + (f - s_pre[r]);
    const int32_t k = A.mcol[e];
    const int64_t ka = A.nrp[k];
    if (A.nrp[k + 1] == ka) {
      A.lofs[e] = 0;
      continue;
    }
    const int o = k - kmin;
    const int u = wpre[o >> 5] + __popc(bits[o >> 5] & ((1u << (o & 31)) - 1u));
    A.lofs[e] = s_off[u] + (int32_t)((int64_t)A.kofs[e] - ka);
  }
  // staged rows by key: each row's rank is the number of smaller keys
  int cls[3] = {0, 0, 0};
  if (t < T && s_row[t] >= 0) {
    const uint64_t my = s_key[t];
    int rank = 0;
    for (int t2 = 0; t2 < T; t2++)
      if (s_row[t2] >= 0 && s_key[t2] < my) rank++;
    const int32_t i = s_row[t];
    A.srows[r0 + rank] = i;
    A.smeta[r0 + rank] = make_int4((int32_t)s_ma[t], mlen, (int32_t)A.nrp[i],
                                   (int32_t)(A.nrp[i + 1] - A.nrp[i]));
    A.row_staged[s_row[t]] = 1;
    cls[my >> 60] = 1;
  }
  block_excl_scan(cls[0], tmp);
  const int n1 = tmp[PL_BS / 64];
  block_excl_scan(cls[1], tmp);
  const int n2 = tmp[PL_BS / 64];
  block_excl_scan(cls[2], tmp);
  const int n4 = tmp[PL_BS / 64];
  if (t == 0) {
    int32_t* ti = A.tinfo + st * TINFO;
    ti[0] = (int32_t)r0;
    ti[1] = n1;
    ti[2] = n2;
    ti[3] = n4;
    ti[4] = (int32_t)run0;
    ti[5] = NR;
    ti[6] = V;
    ti[7] = (int32_t)c;
  }
}

__global__ void k_flag_to_i64(const uint8_t* a, int64_t* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] ? 1 : 0;
}

// ---------------------------------------------------------------------------
// the product
// ---------------------------------------------------------------------------
// Sum of v over the aligned group of eight lanes, in a fixed tree
// ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)), left in every lane of the
// group: exchanges with lane ^ 1 and lane ^ 2 inside quads, then with lane ^ 4
// by row shifts of four (a lane with bit 2 clear takes lane + 4, one with it
// set lane - 4), all on the DPP network.
__device__ __forceinline__ int dpp_xor(int v, int m) {
  if (m == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad 1,0,3,2
  if (m == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad 2,3,0,1
  const int up = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0xF, false);      // row_shl:4
  const int dn = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);      // row_shr:4
  return (threadIdx.x & 4) ? dn : up;
}

__device__ __forceinline__ double dpp_xor(double v, int m) {
  const int2 a = *reinterpret_cast<const int2*>(&v);
  int2 b;
  b.x = dpp_xor(a.x, m);
  b.y = dpp_xor(a.y, m);
  return *reinterpret_cast<const double*>(&b);
}

__device__ __forceinline__ float dpp_xor(float v, int m) {
  return __int_as_float(dpp_xor(__float_as_int(v), m));
}

template <class T>
__device__ __forceinline__ T group8_sum(T v) {
  v = v + dpp_xor(v, 1);
  v = v + dpp_xor(v, 2);
  v = v + dpp_xor(v, 4);
  return v;
}

// One pack: up to eight rows of at most NS slots, eight lanes per row; lane
// l takes the row's M entries l, l + 8, l + 16, l + 24 of each chunk of 32
// and keeps one partial sum per slot over them (ascending); the eight
// partials of a slot are then added in a fixed tree.  Everything a chunk
// needs from device memory (row metadata, M values, LDS offsets, map words,
// and D for the row's dot product) is loaded before any of it is used, and
// the first pack's loads are issued before the workgroup waits for its
// staged Z rows.
constexpr int TK = 4;   // entries per lane per chunk (chunks of 8 * TK)

template <int NS, class TM>
struct PackRegs {
  static constexpr int NP = NS / 8;
  int4 meta;              // first M entry, M length, first pattern entry, slots
  int32_t row;
  bool valid;
  TM m[TK];
  int32_t lo[TK];
  uint32_t w[TK][NP];
  double d[NP];           // D of slots l, l + 8
};

template <int NS, class TM>
__device__ __forceinline__ void pack_load_meta(PackRegs<NS, TM>& R, const int32_t* rows,
                                               const int4* meta, int cnt) {
  const int g = (threadIdx.x & 63) >> 3;
  R.valid = g < cnt;
  R.meta = R.valid ? meta[g] : make_int4(0, 0, 0, 0);
  R.row = R.valid ? rows[g] : 0;
}

// chunk c0 (entries c0 .. c0 + 32) of the row's M entries, and D
template <int NS, class TM>
__device__ __forceinline__ void pack_load_chunk(PackRegs<NS, TM>& R, int c0, const StageArgs& A,
                                                const TM* mval, const uint32_t* nib,
                                                int64_t nstride, const double* D) {
  constexpr int NP = NS / 8;
  const int l = threadIdx.x & 7;
#pragma unroll
  for (int k = 0; k < TK; k++) {
    const int t = c0 + 8 * k + l;
    const bool v = t < R.meta.y;
    const int64_t e = (int64_t)R.meta.x + t;
    R.m[k] = v ? mval[e] : TM(0);
    R.lo[k] = v ? A.lofs[e] : 0;
#pragma unroll
    for (int q = 0; q < NP; q++) R.w[k][q] = v ? nib[(int64_t)q * nstride + e] : 0xFFFFFFFFu;
  }
  if (c0 == 0) {
#pragma unroll
    for (int q = 0; q < NP; q++) {
      const int sl = l + 8 * q;
      R.d[q] = (D && sl < R.meta.w) ? D[(int64_t)R.meta.z + sl] : 0.0;
    }
  }
}

template <int NS, class TM, class TX, class TY>
__device__ __forceinline__ void pack_compute(PackRegs<NS, TM>& R, const StageArgs& A,
                                             const TM* mval, const uint32_t* nib,
                                             int64_t nstride, const TX* Zs, TY* Y,
                                             const double* D, double* rowdot) {
  constexpr int NP = NS / 8;
  const int l = threadIdx.x & 7;
  const int wl = -wave_min_i32(-R.meta.y);   // longest row of the pack (uniform)
  const int nis = -wave_min_i32(-R.meta.w);  // most slots in the pack (uniform)
  TM acc[NS];
#pragma unroll
  for (int s = 0; s < NS; s++) acc[s] = TM(0);
  for (int c0 = 0; c0 < wl; c0 += 8 * TK) {
    if (c0) pack_load_chunk<NS, TM>(R, c0, A, mval, nib, nstride, D);
#pragma unroll
    for (int k = 0; k < TK; k++) {
      if (c0 + 8 * k < wl) {
#pragma unroll
        for (int s = 0; s < NS; s++) {
          if (s < nis) {
            const uint32_t f = (R.w[k][s >> 3] >> (4 * (s & 7))) & 0xFu;
            const bool hit = f != 0xFu;
            const TX xl = Zs[hit ? R.lo[k] + s + (int)f : 0];
            acc[s] = fma(R.m[k], (TM)(hit ? xl : TX(0)), acc[s]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NS; s++)
    if (s < nis) acc[s] = group8_sum(acc[s]);
  // lane l writes slots l, l + 8 (every lane of the group holds every sum)
  double pr = 0.0;
#pragma unroll
  for (int q = 0; q < NP; q++) {
    const int sl = l + 8 * q;
    TM a = acc[0];
#pragma unroll
    for (int u = 1; u < NS; u++)
      if (u == sl) a = acc[u];
    if (R.valid && sl < R.meta.w) {
      Y[(int64_t)R.meta.z + sl] = (TY)a;
      pr = pr + R.d[q] * (double)a;
    }
  }
  if (rowdot) {
    // <D, Y> of the row: per lane over its slots, then the fixed tree
    pr = group8_sum(pr);
    if (R.valid && l == 0) rowdot[R.row] = pr;
  }
}

template <class TM, class TX, class TY>
__global__ __launch_bounds__(64 * TILE_WAVES) void k_spmm_tile(StageArgs A, const int64_t* mrp,
                                                              const TM* mval,
                                                              const uint32_t* nib, int64_t nnzm,
                                                              const int64_t* nrp, const TX* X,
                                                              TY* Y, const double* D,
                                                              double* rowdot) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t st = xcd_block(blockIdx.x, gridDim.x);
  const int32_t* ti = A.tinfo + st * TINFO;
  const int32_t row0 = ti[0], n1 = ti[1], n2 = ti[2], run0 = ti[4], nrun = ti[5];
  TX* Zs = reinterpret_cast<TX*>(smem);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p1 = (n1 + 7) >> 3, p2 = (n2 + 7) >> 3;
  const int32_t* rows = A.srows + row0;
  const int4* meta = A.smeta + row0;
  // the wave's first pack: its loads go out before the staging wait
  PackRegs<8, TM> R8;
  PackRegs<16, TM> R16;
  int p = wv;
  if (p < p1) {
    pack_load_meta<8, TM>(R8, rows + 8 * p, meta + 8 * p, n1 - 8 * p);
    pack_load_chunk<8, TM>(R8, 0, A, mval, nib, nnzm, D);
  } else if (p < p1 + p2) {
    const int a = n1 + 8 * (p - p1);
    pack_load_meta<16, TM>(R16, rows + a, meta + a, n1 + n2 - a);
    pack_load_chunk<16, TM>(R16, 0, A, mval, nib, nnzm, D);
  }
  // the tile's Z rows: each wave copies whole runs, lanes along the run
  for (int q = wv; q < nrun; q += TILE_WAVES) {
    const TX* src = X + A.rg[run0 + q];
    TX* dst = Zs + A.rl[run0 + q];
    const int len = A.rn[run0 + q];
    int v = lane;
    for (; v + 192 < len; v += 256) {
      const TX a0 = src[v], a1 = src[v + 64], a2 = src[v + 128], a3 = src[v + 192];
      dst[v] = a0;
      dst[v + 64] = a1;
      dst[v + 128] = a2;
      dst[v + 192] = a3;
    }
    for (; v < len; v += 64) dst[v] = src[v];
  }
  __syncthreads();
  for (; p < p1 + p2; p += TILE_WAVES) {
    if (p < p1) {
      if (p != wv) {
        pack_load_meta<8, TM>(R8, rows + 8 * p, meta + 8 * p, n1 - 8 * p);
        pack_load_chunk<8, TM>(R8, 0, A, mval, nib, nnzm, D);
      }
      pack_compute<8, TM, TX, TY>(R8, A, mval, nib, nnzm, Zs, Y, D, rowdot);
    } else {
      const int a = n1 + 8 * (p - p1);
      if (p != wv) {
        pack_load_meta<16, TM>(R16, rows + a, meta + a, n1 + n2 - a);
        pack_load_chunk<16, TM>(R16, 0, A, mval, nib, nnzm, D);
      }
      pack_compute<16, TM, TX, TY>(R16, A, mval, nib, nnzm, Zs, Y, D, rowdot);
    }
  }
}

}  // namespace

void stage_plan(EminWork& w, const Csr& M, const int64_t* nrp, const uint8_t* elig,
                const double* xyz, const int32_t* xmap, int dim, hipStream_t s, Arena& ar) {
  StagePlan& P = w.stage;
  P = StagePlan{};
  const int64_t n = w.n;
  if (n == 0 || w.nnz == 0 || M.nnz == 0) return;
  if (M.nnz >= INT32_MAX || w.nnz >= INT32_MAX) return;   // (32-bit offsets in the plan)
  if (xyz && (dim < 1 || dim > 3)) throw Error(EMIN_ERR_ARG, "tile plan: dimension");
  const TileDims D;
  static_assert(TileDims{}.tmax <= PL_BS, "one row per plan thread");
  // cells: at most 4 n / tgt + 64 with coordinates (the cell grows beyond
  // that), blocks of tgt rows without
  const int64_t ncap = xyz ? 4 * n / D.tgt + 64 : (n + D.tgt - 1) / D.tgt;
  if (ncap >= INT32_MAX) return;
  CellGrid* grid = ar.alloc<CellGrid>(1);
  int32_t* key = ar.alloc<int32_t>(n);
  int64_t* coff = ar.alloc<int64_t>(ncap + 1);
  int32_t* cur = ar.alloc<int32_t>(ncap);
  int32_t* csort = ar.alloc<int32_t>(n);
  HIP_OK(hipMemsetAsync(coff, 0, sizeof(int64_t) * (ncap + 1), s));
  HIP_OK(hipMemsetAsync(cur, 0, sizeof(int32_t) * ncap, s));
  if (xyz) k_cell_grid<<<1, 1024, 0, s>>>(xyz, xmap, dim, n, D.tgt, ncap, grid);
  k_cell_key<<<nblocks(n, 256), 256, 0, s>>>(xyz, xmap, dim, n, D.tgt, grid, key, coff);
  scan_inclusive(coff + 1, ncap, s, ar);
  k_cell_place<<<nblocks(n, 256), 256, 0, s>>>(key, n, coff, cur, csort);
  uint8_t* flag = ar.alloc<uint8_t>(ncap);
  int64_t* nrun = ar.alloc<int64_t>(ncap);
  int32_t* vmax = ar.alloc<int32_t>(1);
  unsigned long long* cnt = ar.alloc<unsigned long long>(4);
  HIP_OK(hipMemsetAsync(vmax, 0, sizeof(int32_t), s));
  HIP_OK(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), s));
  PlanArgs A{};
  A.D = D;
  A.mrp = M.rowptr;
  A.mcol = M.col;
  A.nrp = nrp;
  A.kofs = w.kofs;
  A.elig = elig;
  A.coff = coff;
  A.csort = csort;
  A.flag = flag;
  A.nrun = nrun;
  A.vmax = vmax;
  A.cnt = cnt;
  const size_t dyn = plan_lds(D);
  allow_lds((const void*)k_tile_plan<0>);
  allow_lds((const void*)k_tile_plan<1>);
  k_tile_plan<0><<<(unsigned)ncap, PL_BS, dyn, s>>>(A);
  int64_t* tix = ar.alloc<int64_t>(ncap);
  k_flag_to_i64<<<nblocks(ncap, 256), 256, 0, s>>>(flag, tix, ncap);
  scan_inclusive(tix, ncap, s, ar);
  scan_inclusive(nrun, ncap, s, ar);
  unsigned long long hc[4];
  int64_t tot_runs = 0;
  int32_t hv = 0;
  HIP_OK(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&tot_runs, nrun + ncap - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&hv, vmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t nt = (int64_t)hc[3];
  if (nt == 0 || tot_runs >= INT32_MAX) return;
  int32_t* tinfo = ar.alloc<int32_t>((size_t)nt * TINFO);
  int32_t* srows = ar.alloc<int32_t>(n);
  int4* smeta = ar.alloc<int4>(n);
  int32_t* rg = ar.alloc<int32_t>(tot_runs);
  int32_t* rl = ar.alloc<int32_t>(tot_runs);
  int32_t* rn = ar.alloc<int32_t>(tot_runs);
  int32_t* lofs = ar.alloc<int32_t>(M.nnz);
  uint8_t* rs = ar.alloc<uint8_t>(n);
  HIP_OK(hipMemsetAsync(rs, 0, (size_t)n, s));
  A.tix = tix;
  A.roff = nrun;
  A.tinfo = tinfo;
  A.srows = srows;
  A.smeta = smeta;
  A.rg = rg;
  A.rl = rl;
  A.rn = rn;
  A.lofs = lofs;
  A.row_staged = rs;
  k_tile_plan<1><<<(unsigned)ncap, PL_BS, dyn, s>>>(A);
  P.dims = D;
  P.ntile = nt;
  P.tinfo = tinfo;
  P.srows = srows;
  P.smeta = smeta;
  P.rg = rg;
  P.rl = rl;
  P.rn = rn;
  P.lofs = lofs;
  P.row_staged = rs;
  P.vmax = hv;
  P.rows = (int64_t)hc[0];
  P.m_entries = (int64_t)hc[1];
  P.p_entries = (int64_t)hc[2];
}

template <class TM, class TX, class TY>
void spmm_stage(const EminWork& w, const int64_t* mrp, const TM* mval, const int64_t* nrp,
                const TX* X, TY* Y, const double* Dv, hipStream_t s, hipEvent_t e0,
                hipEvent_t e1) {
  const StagePlan& P = w.stage;
  if (P.ntile == 0) return;
  StageArgs A;
  A.tinfo = P.tinfo;
  A.srows = P.srows;
  A.smeta = P.smeta;
  A.rg = P.rg;
  A.rl = P.rl;
  A.rn = P.rn;
  A.lofs = P.lofs;
  A.zbytes = (int32_t)(((size_t)P.vmax * sizeof(TX) + 15) & ~size_t(15));

  const size_t lds = (size_t)A.zbytes;
  allow_lds((const void*)k_spmm_tile<TM, TX, TY>);
  if (e0 || e1) {
    hipExtLaunchKernelGGL(k_spmm_tile<TM, TX, TY>, dim3((unsigned)P.ntile), dim3(64 * TILE_WAVES),
                          lds, s, e0, e1, 0, A, mrp, mval, (const uint32_t*)w.nib, w.nnzm, nrp, X,
                          Y, Dv, Dv ? w.rowdot : nullptr);
    HIP_OK(hipGetLastError());
  } else {
    k_spmm_tile<TM, TX, TY><<<(unsigned)P.ntile, 64 * TILE_WAVES, lds, s>>>(
        A, mrp, mval, w.nib, w.nnzm, nrp, X, Y, Dv, Dv ? w.rowdot : nullptr);
  }
}

template void spmm_stage<double, double, double>(const EminWork&, const int64_t*, const double*,
                                                 const int64_t*, const double*, double*,
                                                 const double*, hipStream_t, hipEvent_t,
                                                 hipEvent_t);
template void spmm_stage<float, float, float>(const EminWork&, const int64_t*, const float*,
                                              const int64_t*, const float*, float*, const double*,
                                              hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace emin
