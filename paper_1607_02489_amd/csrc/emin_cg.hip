// sec. 4.3, eq. (min_problem): EMIN-AMG prolongator values by constrained CG
// on trace(P^T M P) over matrices with P's fixed pattern that keep P W_c = W.
//
// Hot kernel: the masked product Q = mask_N(M Z).  G lanes own one row i:
// they split M's row i, and for each k merge the short sorted row k of the
// pattern against row i's columns (held in registers), accumulating per
// output slot; the G partial sums are combined by a fixed xor-butterfly, so
// results are deterministic.  Projection and CG updates are row-local; every
// reduction is a fixed two-level tree (block partials, then one block), and
// the CG scalars (rho, gamma, alpha, beta, energy) never leave the device.
#include "emin_cg.h"
#include "prof.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>

namespace emin {


__device__ __forceinline__ double block_sum(double v, double* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) t += lds[k];
  return t;  // valid on thread 0
}

// W_c = W restricted to the C points; Gram g_i = sum over the row's pattern
// of W_c^2; P0 = W_i W_c / g_i on F rows (1/|N_i| for a 0/1 mode), 1 on C rows
// (G lanes per pattern row; the Gram sum by a butterfly over the group)
template <int G>
__global__ __launch_bounds__(256) void k_emin_init(const int64_t* rp, const int32_t* col,
                                                  int64_t n, const int32_t* cid, const double* W,
                                                  const double* Wc, double* Gm, double* P,
                                                  int32_t* status) {
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t i = (int64_t)blockIdx.x * NG + g;
  if (i >= n) return;
  const int64_t a = rp[i], b = rp[i + 1];
  double gs = 0.0;
  for (int64_t s = a + lane; s < b; s += G) gs = gs + Wc[col[s]] * Wc[col[s]];
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) gs += __shfl_xor(gs, m, G);
  if (lane == 0) Gm[i] = gs;
  if (cid[i] >= 0) {
    for (int64_t s = a + lane; s < b; s += G) P[s] = 1.0;
    return;
  }
  if (gs > 0.0) {
    for (int64_t s = a + lane; s < b; s += G) P[s] = (W[i] * Wc[col[s]]) / gs;
  } else {
    for (int64_t s = a + lane; s < b; s += G) P[s] = 0.0;
    if (lane == 0 && W[i] != 0.0) atomicMax(status, (int32_t)EMIN_ERR_INFEASIBLE);
  }
}

__global__ void k_gather_modes(const double* W, const int32_t* clist, int64_t nc, double* Wc) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) Wc[c] = W[clist[c]];
}

__global__ void k_default_modes(const uint8_t* dir, int64_t n, double* W) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) W[i] = dir ? (dir[i] ? 0.0 : 1.0) : 1.0;
}

// Row-binned masked product: G lanes own one row i whose pattern has at most G
// entries, lane s computing slot s (column j_s).  The group first stages M's
// row i and the pattern-row bounds of its columns k across its lanes (two
// coalesced loads), then walks the k's four at a time: the four pattern rows
// (columns and X values, G entries each) are loaded together, and each lane
// finds j_s among them by a binary search over the lanes.  Every slot sums
// over k in ascending order, so results are deterministic.
template <int G, class TX>
__device__ __forceinline__ TX find_in_group(int32_t js, int32_t c, TX z, bool& hit) {
  int pos = 0;
#pragma unroll
  for (int step = G / 2; step >= 1; step >>= 1) {
    const int32_t cp = __shfl(c, pos + step - 1, G);
    if (cp < js) pos += step;
  }
  const int32_t cf = __shfl(c, pos, G);
  const TX zf = __shfl(z, pos, G);
  hit = (cf == js);
  return zf;
}

template <int G, class TM, class TX, class TY>
__device__ __forceinline__ void spmm_search_rows(int64_t lb, const int32_t* rows, int64_t nrows,
                                                 const int64_t* mrp, const int32_t* mcol,
                                                 const TM* mval, const int64_t* nrp,
                                                 const int32_t* ncol, const TX* X, TY* Y,
                                                 const double* D, double* rowdot) {
  using TA = TM;
  constexpr int NG = SPMM_BS / G;
  constexpr int U = 4;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t r = lb * NG + g;
  if (r < nrows) {
    const int32_t i = rows[r];
    const int64_t na = nrp[i];
    const int ni = (int)(nrp[i + 1] - na);
    const int32_t js = lane < ni ? ncol[na + lane] : INT32_MAX;
    const int64_t ma = mrp[i], mb = mrp[i + 1];
    TA acc = TA(0);
    for (int64_t e0 = ma; e0 < mb; e0 += G) {
      const int64_t e = e0 + lane;
      const bool ev = e < mb;
      const int32_t kk = ev ? mcol[e] : 0;
      const TA mvv = ev ? (TA)mval[e] : TA(0);
      const int64_t ka = ev ? nrp[kk] : 0;
      const int len = ev ? (int)(nrp[kk + 1] - ka) : 0;
      const int cnt = (int)((mb - e0) < G ? (mb - e0) : G);
      for (int q0 = 0; q0 < cnt; q0 += U) {
        int32_t c[U];
        TX z[U];
        TA m[U];
        int64_t a[U];
        int l[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int q = q0 + u;
          const bool qv = q < cnt;
          a[u] = __shfl(ka, q, G);
          l[u] = qv ? __shfl(len, q, G) : 0;
          m[u] = __shfl(mvv, q, G);
          const int64_t t = a[u] + lane;
          c[u] = lane < l[u] ? ncol[t] : INT32_MAX;
          z[u] = lane < l[u] ? X[t] : TX(0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          bool hit;
          TX zf = find_in_group<G, TX>(js, c[u], z[u], hit);
          for (int off = G; off < l[u]; off += G) {   // pattern row k longer than G (uniform)
            const int64_t t = a[u] + off + lane;
            const int32_t cc = off + lane < l[u] ? ncol[t] : INT32_MAX;
            const TX zz = off + lane < l[u] ? X[t] : TX(0);
            bool h2;
            const TX z2 = find_in_group<G, TX>(js, cc, zz, h2);
            if (h2 && !hit) { zf = z2; hit = true; }
          }
          if (hit) acc = fma(m[u], (TA)zf, acc);
        }
      }
    }
    if (lane < ni) Y[na + lane] = (TY)acc;
    if (rowdot) {
      // <D, Y> of the row, summed in slot order by lane 0
      const double pr = lane < ni ? D[na + lane] * (double)acc : 0.0;
      double sum = 0.0;
      for (int t = 0; t < ni; t++) sum = sum + __shfl(pr, t, G);
      if (lane == 0) rowdot[i] = sum;
    }
  }
}

// Precomputed intersection maps.  For an M entry (i,k), slot s of N_i meets
// column N_i[s] in row k at position pos(s) (or nowhere).  When row i has at
// most 32 slots and, over all its M entries, the offsets pos(s) - s of each
// entry span at most 14, the map of entry e is stored as one base offset into
// the pattern values, kofs[e] = nrp[k] + min(pos(s) - s), and one 4-bit field
// per slot, pos(s) - s - min or 15 for "no match", packed eight to a 32-bit
// word (plane q of the word array holds slots 8q..8q+7).  Rows that do not
// fit are marked ineligible and keep the searching kernel.
template <int G>
__global__ __launch_bounds__(256) void k_spmm_maps(const int64_t* mrp, const int32_t* mcol,
                                                  const int64_t* nrp, const int32_t* ncol,
                                                  int64_t n, int64_t nnzm, int nplanes,
                                                  int32_t* kofs, uint32_t* nib, uint8_t* elig) {
  // G lanes per row i, lane t taking M entries t, t + G, ...
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t i = (int64_t)blockIdx.x * (256 / G) + g;
  if (i >= n) return;   // whole group
  const int64_t na = nrp[i], nb = nrp[i + 1];
  const int ni = (int)(nb - na);
  const int planes = ni <= 8 ? 1 : (ni <= 16 ? 2 : 4);
  bool ok = ni <= 32 && planes <= nplanes;   // this lane's entries all fit
  for (int64_t e = mrp[i] + lane; e < mrp[i + 1]; e += G) {
    const int32_t k = mcol[e];
    const int64_t ka = nrp[k], kb = nrp[k + 1];
    uint32_t w[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    int64_t base = 0;
    if (ok) {
      // pass 1: range of pos(s) - s
      int64_t lo = INT64_MAX, hi = INT64_MIN;
      for (int pass = 0; pass < 2 && ok; pass++) {
        int64_t a = na, b = ka;
        while (a < nb && b < kb) {
          const int32_t ca = ncol[a], cb = ncol[b];
          if (ca < cb) a++;
          else if (cb < ca) b++;
          else {
            const int64_t off = (b - ka) - (a - na);
            if (pass == 0) {
              lo = off < lo ? off : lo;
              hi = off > hi ? off : hi;
            } else {
              const int sl = (int)(a - na);
              const uint32_t f = (uint32_t)(off - lo);
              w[sl >> 3] &= ~(0xFu << (4 * (sl & 7)));
              w[sl >> 3] |= f << (4 * (sl & 7));
            }
            a++;
            b++;
          }
        }
        if (pass == 0) {
          if (lo == INT64_MAX) break;          // no common column: all fields 15
          if (hi - lo > 14) ok = false;
        }
      }
      base = lo == INT64_MAX ? 0 : lo;
    }
    const int64_t ko = ka + base;
    if (ko < INT32_MIN + 64 || ko > INT32_MAX - 64) ok = false;
    kofs[e] = (int32_t)(ok ? ko : 0);
    for (int q = 0; q < nplanes; q++) nib[(int64_t)q * nnzm + e] = w[q];
  }
  const bool all = group_ballot<G>(!ok) == 0ull;
  if (lane == 0) elig[i] = all ? 1 : 0;
}

// Masked product on the intersection maps: G lanes (G >= |N_i|) own row i,
// lane s computing slot s.  The group copies M's row (values, base offsets,
// map words) through an LDS window with coalesced loads; then for each entry
// lane s reads its 4-bit field and, on a match, gathers exactly one pattern
// value, X[kofs + s + field].  No searching and no cross-lane traffic;
// per-slot sums run over k in order (deterministic).  The inner loop has no
// branches: the trip count is the longest row of the wave (shorter rows are
// padded with empty maps), a missing match gathers X[0] and adds m * 0, and
// four entries are read from the window with one 16-byte LDS load per array.
template <int G>
struct MapWin {
  static constexpr int NG = SPMM_BS / G;
  static constexpr int WG = 64 / G;                 // groups per wave
  static constexpr int NP = G <= 8 ? 1 : G / 8;     // map planes of a row
  static constexpr int CH = G <= 4 ? 16 : 32;       // window entries per group
};

template <int G, class TM>
constexpr int map_wave_smem() {
  return MapWin<G>::WG * MapWin<G>::CH * (int)(sizeof(TM) + 4 + 4 * MapWin<G>::NP);
}

// LDS of one wave's windows (the largest over the map classes) and of a block
template <class TM>
constexpr int spmm_wave_smem() {
  constexpr int a = map_wave_smem<4, TM>(), b = map_wave_smem<8, TM>(),
                c = map_wave_smem<16, TM>(), d = map_wave_smem<32, TM>();
  constexpr int ab = a > b ? a : b, cd = c > d ? c : d;
  return ((ab > cd ? ab : cd) + 15) & ~15;
}

template <class TM>
constexpr int spmm_smem() {
  return (SPMM_BS / 64) * spmm_wave_smem<TM>();
}

template <class T> struct Vec4;
template <> struct Vec4<double> {
  double v[4];
  __device__ __forceinline__ void load(const double* p) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};
template <> struct Vec4<float> {
  float v[4];
  __device__ __forceinline__ void load(const float* p) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
};

template <int G, int UB, class TM, class TX, class TY>
__device__ __forceinline__ void spmm_map_rows(int64_t lb, const int32_t* rows, int64_t nrows,
                                              const int64_t* mrp, const TM* mval,
                                              const int32_t* kofs, const uint32_t* nib,
                                              int64_t nnzm, const int64_t* nrp, const TX* X,
                                              TY* Y, const double* D, double* rowdot,
                                              unsigned char* smem) {
  using TA = TM;
  using W = MapWin<G>;
  constexpr int NG = W::NG, NP = W::NP, CH = W::CH;
  // each wave owns its own LDS region (its groups' windows): the layout of
  // one wave never depends on another wave's row class
  constexpr int WG = W::WG;
  unsigned char* wbase = smem + (threadIdx.x >> 6) * spmm_wave_smem<TM>();
  TM* s_m = reinterpret_cast<TM*>(wbase);
  int32_t* s_k = reinterpret_cast<int32_t*>(s_m + WG * CH);
  uint32_t* s_w = reinterpret_cast<uint32_t*>(s_k + WG * CH);   // [NP][WG*CH]
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int gi = (threadIdx.x & 63) / G;   // group within the wave
  const int64_t r = lb * NG + g;
  const int q = lane >> 3, sh = 4 * (lane & 7);
  TM* gm = s_m + gi * CH;
  int32_t* gk = s_k + gi * CH;
  const uint32_t* gw = s_w + q * (WG * CH) + gi * CH;
  // rows past the class end join the wave's loops as empty rows
  const bool valid = r < nrows;
  const int32_t i = valid ? rows[r] : 0;
  const int64_t na = valid ? nrp[i] : 0;
  const int ni = valid ? (int)(nrp[i + 1] - na) : 0;
  const int64_t ma = valid ? mrp[i] : 0;
  const int len = valid ? (int)(mrp[i + 1] - ma) : 0;
  const int wl = -wave_min_i32(-len);   // longest row of the wave (uniform)
  const double dv = (rowdot && lane < ni) ? D[na + lane] : 0.0;
  TA acc = TA(0);
  for (int c0 = 0; c0 < wl; c0 += CH) {
    const int cw = ((wl - c0 < CH ? wl - c0 : CH) + UB - 1) & ~(UB - 1);   // uniform
    for (int t = lane; t < cw; t += G) {
      const bool v = c0 + t < len;
      const int64_t e = ma + c0 + t;
      gm[t] = v ? mval[e] : TM(0);
      gk[t] = v ? kofs[e] : 0;
#pragma unroll
      for (int p = 0; p < NP; p++)
        s_w[p * (WG * CH) + gi * CH + t] = v ? nib[(int64_t)p * nnzm + e] : 0xFFFFFFFFu;
    }
    // the group lies inside one wave: order its LDS writes before the reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // UB entries per step: every gather of the step is issued before the
    // first multiply-add, so a lane has UB loads in flight
    for (int t = 0; t < cw; t += UB) {
      TX x[UB];
#pragma unroll
      for (int q = 0; q < UB; q += 4) {
        const uint4 w4 = *reinterpret_cast<const uint4*>(gw + t + q);
        const int4 k4 = *reinterpret_cast<const int4*>(gk + t + q);
        const uint32_t wv[4] = {w4.x, w4.y, w4.z, w4.w};
        const int32_t kv[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const uint32_t f = (wv[u] >> sh) & 0xFu;
          const bool hit = f != 0xFu;
          // 32-bit byte offset (a pattern of fewer than 2^29 entries): the
          // load takes X as a scalar base plus one vector offset
          const uint32_t off = (uint32_t)(hit ? kv[u] + lane + (int)f : 0) * (uint32_t)sizeof(TX);
          const TX xl = *reinterpret_cast<const TX*>(reinterpret_cast<const char*>(X) + off);
          x[q + u] = hit ? xl : TX(0);
        }
      }
#pragma unroll
      for (int q = 0; q < UB; q += 4) {
        Vec4<TM> m4;
        m4.load(gm + t + q);
#pragma unroll
        for (int u = 0; u < 4; u++) acc = fma(m4.v[u], (TA)x[q + u], acc);
      }
    }
    // every lane is done with the window before the next pass refills it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (valid) {
    if (lane < ni) Y[na + lane] = (TY)acc;
    if (rowdot) {
      // <D, Y> of the row, summed in slot order by lane 0
      const double pr = lane < ni ? dv * (double)acc : 0.0;
      double sum = 0.0;
      for (int t = 0; t < ni; t++) sum = sum + __shfl(pr, t, G);
      if (lane == 0) rowdot[i] = sum;
    }
  }
}

// The whole masked product in one launch: block ranges serve the row classes
// (map rows with G = 4, 8, 16, 32 lanes, then searched rows with G = 4 ...
// 64).  Every class has a multiple of 8 blocks.  With xcd_split each XCD
// (which receives the hardware blocks x, x+8, ...) takes the x-th eighth of
// every class, so the load is balanced across XCDs and each XCD works on
// contiguous rows; otherwise each XCD takes one contiguous eighth of the grid.
template <class TM, class TX, class TY>
__global__ __launch_bounds__(SPMM_BS) void k_spmm(SpmmSched S, const int64_t* mrp,
                                              const int32_t* mcol, const TM* mval,
                                              const int32_t* kofs, const uint32_t* nib,
                                              int64_t nnzm, const int64_t* nrp,
                                              const int32_t* ncol, const TX* X, TY* Y,
                                              const double* D, double* rowdot) {
  __shared__ __align__(16) unsigned char smem[spmm_smem<TM>()];
  int ty = 0;
  int64_t lb;
  if (S.xcd_split == XCD_MERGED) {
    const int32_t m = S.bmap[xcd_block(blockIdx.x, gridDim.x)];
    ty = m >> 27;
    lb = m & ((1 << 27) - 1);
  } else if (S.xcd_split == XCD_BY_CLASS) {
    const int64_t x = blockIdx.x & 7, j = blockIdx.x >> 3;
#pragma unroll
    for (int t = 1; t < SPMM_NT; t++) ty += j >= (S.blk_off[t] >> 3) ? 1 : 0;
    const int64_t q = (S.blk_off[ty + 1] - S.blk_off[ty]) >> 3;
    lb = x * q + (j - (S.blk_off[ty] >> 3));
  } else {
    // one contiguous eighth of the whole grid per XCD
    const int64_t gb = xcd_block(blockIdx.x, gridDim.x);
#pragma unroll
    for (int t = 1; t < SPMM_NT; t++) ty += gb >= S.blk_off[t] ? 1 : 0;
    lb = gb - S.blk_off[ty];
  }
  const int32_t* rows = S.rows + S.row_off[ty];
  const int64_t nr = S.row_off[ty + 1] - S.row_off[ty];
  double* rd = D ? rowdot : nullptr;
  if (S.unroll >= 16) {
    switch (ty) {
      case 0: spmm_map_rows<4, 16>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); return;
      case 1: spmm_map_rows<8, 16>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); return;
      case 2: spmm_map_rows<16, 16>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); return;
      case 3: spmm_map_rows<32, 16>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); return;
      default: break;
    }
  }
  switch (ty) {
    case 0: spmm_map_rows<4, 4>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); break;
    case 1: spmm_map_rows<8, 4>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); break;
    case 2: spmm_map_rows<16, 4>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); break;
    case 3: spmm_map_rows<32, 4>(lb, rows, nr, mrp, mval, kofs, nib, nnzm, nrp, X, Y, D, rd, smem); break;
    case 4: spmm_search_rows<4>(lb, rows, nr, mrp, mcol, mval, nrp, ncol, X, Y, D, rd); break;
    case 5: spmm_search_rows<8>(lb, rows, nr, mrp, mcol, mval, nrp, ncol, X, Y, D, rd); break;
    case 6: spmm_search_rows<16>(lb, rows, nr, mrp, mcol, mval, nrp, ncol, X, Y, D, rd); break;
    case 7: spmm_search_rows<32>(lb, rows, nr, mrp, mcol, mval, nrp, ncol, X, Y, D, rd); break;
    default: spmm_search_rows<64>(lb, rows, nr, mrp, mcol, mval, nrp, ncol, X, Y, D, rd); break;
  }
}

// <D, Y> over all rows from the per-row values, in a fixed tree: block b sums
// rows [1024 b, 1024 b + 1024) (four per thread in order, then the block
// tree); the result does not depend on how the product was scheduled.
__global__ __launch_bounds__(256) void k_rowsum(const double* rowdot, int64_t n, double* part) {
  __shared__ double lds[4];
  const int64_t b0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  double v = 0.0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int64_t i = b0 + 256 * j;
    if (i < n) v = v + rowdot[i];
  }
  const double t = block_sum(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The row-local kernels below take G lanes per pattern row (a wave covers
// 64 / G consecutive rows, so its loads are consecutive entries of the
// pattern arrays): lane t holds entries t, t + G, ... of the row, the
// projection's dot product is the lanes' sums added by a butterfly over the
// group, and the block partials of <R,R> (and <P,MP>) are summed in a fixed
// tree.

// R = -Pi(MP), Z = R, partial <R,R>
template <int G>
__global__ __launch_bounds__(256) void k_init_r(const int64_t* rp, const int32_t* col, int64_t n,
                                               const int32_t* cid, const double* Wc,
                                               const double* Gm, const double* MP, double* R,
                                               double* Z, double* part) {
  __shared__ double lds[4];
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t i = (int64_t)blockIdx.x * NG + g;
  double rr = 0.0;
  if (i < n) {
    const int64_t a = rp[i], b = rp[i + 1];
    if (cid[i] >= 0) {
      for (int64_t s = a + lane; s < b; s += G) { R[s] = 0.0; Z[s] = 0.0; }
    } else {
      double dot = 0.0;
      for (int64_t s = a + lane; s < b; s += G) dot = dot + (-MP[s]) * Wc[col[s]];
#pragma unroll
      for (int m = G / 2; m >= 1; m >>= 1) dot += __shfl_xor(dot, m, G);
      const double gi = Gm[i];
      const double f = gi > 0.0 ? dot / gi : 0.0;
      for (int64_t s = a + lane; s < b; s += G) {
        const double r = -MP[s] - f * Wc[col[s]];
        R[s] = r;
        Z[s] = r;
        rr += r * r;
      }
    }
  }
  const double t = block_sum(rr, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// P += alpha Z; R -= alpha Pi(Q); partial <R,R>; with the energy trace also
// MP += alpha Q and partial <P, MP>
template <int G, class TQ>
__global__ __launch_bounds__(256) void k_update(const int64_t* rp, const int32_t* col, int64_t n,
                                               const int32_t* cid, const double* Wc,
                                               const double* Gm, const double* Z, const TQ* Q,
                                               double* P, double* R, double* MP,
                                               const CgScalars* sc, double* part,
                                               double* part_e) {
  __shared__ double lds[4];
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t i = (int64_t)blockIdx.x * NG + g;
  const double alpha = sc->alpha;
  double rr = 0.0, ee = 0.0;
  if (i < n) {
    const int64_t a = rp[i], b = rp[i + 1];
    if (cid[i] < 0) {
      double dot = 0.0;
      for (int64_t s = a + lane; s < b; s += G) dot = dot + (double)Q[s] * Wc[col[s]];
#pragma unroll
      for (int m = G / 2; m >= 1; m >>= 1) dot += __shfl_xor(dot, m, G);
      const double gi = Gm[i];
      const double f = gi > 0.0 ? dot / gi : 0.0;
      for (int64_t s = a + lane; s < b; s += G) {
        const double q = (double)Q[s];
        const double pq = q - f * Wc[col[s]];
        const double p = P[s] + alpha * Z[s];
        const double r = R[s] - alpha * pq;
        P[s] = p;
        R[s] = r;
        rr += r * r;
        if (MP) {
          const double mp = MP[s] + alpha * q;
          MP[s] = mp;
          ee += p * mp;
        }
      }
    } else if (MP) {
      for (int64_t s = a + lane; s < b; s += G) {
        const double mp = MP[s] + alpha * (double)Q[s];
        MP[s] = mp;
        ee += P[s] * mp;
      }
    }
  }
  double t = block_sum(rr, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
  if (part_e) {
    t = block_sum(ee, lds);
    if (threadIdx.x == 0) part_e[blockIdx.x] = t;
  }
}

// lanes per row of the row-local kernels: about the average pattern row
static int update_lanes(int64_t n, int64_t nnz) {
  const double avg = n ? (double)nnz / (double)n : 1.0;
  int g = 4;
  while (g < 32 && g < 0.8 * avg) g <<= 1;
  return g;
}

static void launch_emin_init(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz,
                             const int32_t* cid, const double* W, const double* Wc, double* Gm,
                             double* P, int32_t* status, hipStream_t s) {
  switch (update_lanes(n, nnz)) {
    case 4: k_emin_init<4><<<nblocks(n, 64), 256, 0, s>>>(rp, col, n, cid, W, Wc, Gm, P, status); break;
    case 8: k_emin_init<8><<<nblocks(n, 32), 256, 0, s>>>(rp, col, n, cid, W, Wc, Gm, P, status); break;
    case 16: k_emin_init<16><<<nblocks(n, 16), 256, 0, s>>>(rp, col, n, cid, W, Wc, Gm, P, status); break;
    default: k_emin_init<32><<<nblocks(n, 8), 256, 0, s>>>(rp, col, n, cid, W, Wc, Gm, P, status); break;
  }
}

template <int G>
static int64_t launch_init_r(const EminWork& w, const int64_t* nrp, const int32_t* ncol,
                             const int32_t* cid, hipStream_t s) {
  const int64_t nb = nblocks(w.n, 256 / G);
  k_init_r<G><<<(unsigned)nb, 256, 0, s>>>(nrp, ncol, w.n, cid, w.Wc, w.G, w.MP, w.R, w.Z, w.part);
  return nb;
}

template <int G>
static int64_t launch_update(const EminWork& w, const int64_t* nrp, const int32_t* ncol,
                             const int32_t* cid, double* P, bool energy, bool mixed,
                             hipStream_t s) {
  const int64_t nb = nblocks(w.n, 256 / G);
  if (mixed)
    k_update<G, float><<<(unsigned)nb, 256, 0, s>>>(nrp, ncol, w.n, cid, w.Wc, w.G, w.Z, w.Qf, P,
                                                    w.R, energy ? w.MP : nullptr, w.sc, w.part,
                                                    energy ? w.part_e : nullptr);
  else
    k_update<G, double><<<(unsigned)nb, 256, 0, s>>>(nrp, ncol, w.n, cid, w.Wc, w.G, w.Z, w.Q, P,
                                                     w.R, energy ? w.MP : nullptr, w.sc, w.part,
                                                     energy ? w.part_e : nullptr);
  return nb;
}

static int64_t init_r(const EminWork& w, const int64_t* nrp, const int32_t* ncol,
                      const int32_t* cid, hipStream_t s) {
  switch (update_lanes(w.n, w.nnz)) {
    case 4: return launch_init_r<4>(w, nrp, ncol, cid, s);
    case 8: return launch_init_r<8>(w, nrp, ncol, cid, s);
    case 16: return launch_init_r<16>(w, nrp, ncol, cid, s);
    default: return launch_init_r<32>(w, nrp, ncol, cid, s);
  }
}

static int64_t cg_update(const EminWork& w, const int64_t* nrp, const int32_t* ncol,
                         const int32_t* cid, double* P, bool energy, bool mixed, hipStream_t s) {
  switch (update_lanes(w.n, w.nnz)) {
    case 4: return launch_update<4>(w, nrp, ncol, cid, P, energy, mixed, s);
    case 8: return launch_update<8>(w, nrp, ncol, cid, P, energy, mixed, s);
    case 16: return launch_update<16>(w, nrp, ncol, cid, P, energy, mixed, s);
    default: return launch_update<32>(w, nrp, ncol, cid, P, energy, mixed, s);
  }
}

// Z = R + beta Z (and the FP32 copy used by the mixed-precision product)
__global__ void k_zupd(const double* R, double* Z, float* Zf, int64_t nnz, const CgScalars* sc) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const double z = R[e] + sc->beta * Z[e];
  Z[e] = z;
  if (Zf) Zf[e] = (float)z;
}

__global__ void k_to_float(const double* a, float* b, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}

enum FinMode { FIN_E0 = 0, FIN_RHO0 = 1, FIN_GAMMA = 2, FIN_RHO = 3, FIN_E = 4 };

// Sum of block partials in a fixed order, then the CG scalar logic:
// gamma <= 0 with rho > 0 is a breakdown; rho == 0 stops early.
__global__ __launch_bounds__(1024) void k_finalize(const double* part, int np, CgScalars* sc,
                                                   int mode, int it, double* rep_e,
                                                   double* rep_rho, double* rep_gamma,
                                                   int32_t* rep_its, int32_t* rep_status) {
  __shared__ double lds[16];
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) v += part[k];
  const double tot = block_sum(v, lds);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case FIN_E0:
      if (rep_e) rep_e[0] = tot;
      break;
    case FIN_RHO0:
      sc->rho = tot;
      sc->alpha = 0.0;
      sc->beta = 0.0;
      sc->stop = 0;
      sc->its = 0;
      if (rep_rho) rep_rho[0] = tot;
      break;
    case FIN_GAMMA:
      if (rep_gamma) rep_gamma[it] = tot;
      if (sc->stop || sc->rho == 0.0) {
        sc->stop = 1;
        sc->alpha = 0.0;
      } else if (!(tot > 0.0)) {
        sc->stop = 1;
        sc->alpha = 0.0;
        if (rep_status) atomicMax(rep_status, (int32_t)EMIN_ERR_BREAKDOWN);
      } else {
        sc->alpha = sc->rho / tot;
        sc->its += 1;
        if (rep_its) *rep_its = sc->its;
      }
      break;
    case FIN_RHO:
      if (sc->stop) {
        sc->beta = 0.0;
      } else {
        sc->beta = tot / sc->rho;
        sc->rho = tot;
        if (rep_rho) rep_rho[it + 1] = tot;
      }
      break;
    case FIN_E:
      if (!sc->stop && rep_e) rep_e[it + 1] = tot;
      break;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void EminWork::allocate(int64_t n_, int64_t nnz_, int64_t nc_, Arena& ar, bool mixed) {
  n = n_;
  nnz = nnz_;
  nc = nc_;
  G = ar.alloc<double>(n);
  Wc = ar.alloc<double>(nc);
  Wdef = ar.alloc<double>(n);
  R = ar.alloc<double>(nnz);
  Z = ar.alloc<double>(nnz);
  Q = ar.alloc<double>(nnz);
  MP = ar.alloc<double>(nnz);
  Zf = ar.alloc<float>(nnz);
  Qf = ar.alloc<float>(nnz);
  (void)mixed;
  // enough for every grid used (the masked product pads each row class to a
  // multiple of 8 blocks)
  const int64_t np = 2 * (int64_t)nblocks(n, 4) + 16 + 8 * SPMM_NT;
  part = ar.alloc<double>(np);
  part_e = ar.alloc<double>(np);
  rowdot = ar.alloc<double>(n);
  sc = ar.alloc<CgScalars>(1);
}

// Row classes: -1 for an empty pattern row, 0..3 for map rows with
// G = 4..32 lanes, 4..8 for searched rows with G = 4..64.  gshift moves a
// row to a class with 2^gshift times more lanes than its length needs.
__device__ __forceinline__ int spmm_class(int64_t len, bool map, int gshift) {
  if (len <= 0) return -1;
  int b = len <= 4 ? 0 : (len <= 8 ? 1 : (len <= 16 ? 2 : (len <= 32 ? 3 : 4)));
  b += gshift;
  if (b > 4) b = 4;
  return (map && b <= 3) ? b : 4 + b;
}

// per block (256 rows) and class, the number of rows; class-major
__global__ __launch_bounds__(256) void k_sched_count(const int64_t* nrp, const uint8_t* elig,
                                                    const uint8_t* skip, int64_t n, int maps,
                                                    int gshift, int64_t* bc, int64_t nb) {
  __shared__ int cnt[SPMM_NT];
  if (threadIdx.x < SPMM_NT) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = (i < n && !(skip && skip[i]))
                    ? spmm_class(nrp[i + 1] - nrp[i], maps && elig[i], gshift) : -1;
  if (c >= 0) atomicAdd(&cnt[c], 1);
  __syncthreads();
  if (threadIdx.x < SPMM_NT) bc[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// stable placement: class-major, ascending row index within a class
// (inclusive scan of the class-major block counts gives each block's start)
__global__ __launch_bounds__(256) void k_sched_place(const int64_t* nrp, const uint8_t* elig,
                                                    const uint8_t* skip, int64_t n, int maps,
                                                    int gshift, const int64_t* incl, int64_t nb,
                                                    int32_t* rows) {
  __shared__ int wc[4][SPMM_NT];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = (i < n && !(skip && skip[i]))
                    ? spmm_class(nrp[i + 1] - nrp[i], maps && elig[i], gshift) : -1;
  const uint64_t below = (1ull << lane) - 1ull;
  uint64_t mine = 0;
  for (int q = 0; q < SPMM_NT; q++) {
    const uint64_t m = __ballot(c == q);
    if (lane == 0) wc[w][q] = __popcll(m);
    if (c == q) mine = m;
  }
  __syncthreads();
  if (c < 0) return;
  const int64_t k = (int64_t)c * nb + blockIdx.x;
  int64_t pos = k ? incl[k - 1] : 0;   // where this block's rows of class c start
  for (int v = 0; v < w; v++) pos += wc[v][c];
  rows[pos + __popcll(mine & below)] = (int32_t)i;
}

// XCD_MERGED order: block lb of class c goes to slot lb + the number of
// blocks of the other classes whose first row comes before its own (ties by
// class); padding blocks (no rows) sort last.  The first rows of a class's
// blocks ascend, so each count is a binary search.
struct MergeArgs {
  const int32_t* rows;
  int64_t row_off[SPMM_NT + 1];
  int64_t blk_off[SPMM_NT + 1];
};

__device__ __forceinline__ int64_t first_row(const MergeArgs& A, int c, int64_t lb) {
  const int G = 4 << (c < 4 ? c : c - 4);
  const int64_t r = A.row_off[c] + lb * (SPMM_BS / G);
  return r < A.row_off[c + 1] ? (int64_t)A.rows[r] : INT64_MAX;
}

__global__ void k_sched_merge(MergeArgs A, int32_t* bmap) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.blk_off[SPMM_NT]) return;
  int c = 0;
  while (c + 1 < SPMM_NT && b >= A.blk_off[c + 1]) c++;
  const int64_t lb = b - A.blk_off[c];
  const int64_t key = first_row(A, c, lb);
  int64_t pos = lb;
  for (int c2 = 0; c2 < SPMM_NT; c2++) {
    if (c2 == c) continue;
    // blocks of c2 before (key, c): first row < key, or == key with c2 < c
    int64_t lo = 0, hi = A.blk_off[c2 + 1] - A.blk_off[c2];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      const int64_t k2 = first_row(A, c2, mid);
      if (k2 < key || (k2 == key && c2 < c)) lo = mid + 1; else hi = mid;
    }
    pos += lo;
  }
  bmap[pos] = (int32_t)((c << 27) | (int32_t)lb);
}

__global__ void k_sched_totals(const int64_t* incl, int64_t nb, int64_t* tot) {
  const int c = threadIdx.x;
  if (c < SPMM_NT) tot[c] = incl[(int64_t)(c + 1) * nb - 1];
}

// Schedule of the masked product under one set of options: one counting
// kernel, one scan, one placement kernel, one read-back of the class ends.
static void build_sched(const EminWork& w, const int64_t* nrp, const uint8_t* elig, SchedOpts o,
                        SpmmSched& S, hipStream_t s, Arena& ar) {
  const int64_t n = w.n;
  const int64_t nb = n ? (int64_t)nblocks(n, 256) : 0;
  int64_t tot[SPMM_NT] = {};
  int32_t* rows = ar.alloc<int32_t>(n);
  if (n) {
    int64_t* bc = ar.alloc<int64_t>((size_t)SPMM_NT * nb);
    int64_t* dtot = ar.alloc<int64_t>(SPMM_NT);
    // rows of staged blocks are the staged kernel's
    const uint8_t* skip = (o.stage && w.stage.ntile) ? w.stage.row_staged : nullptr;
    k_sched_count<<<(unsigned)nb, 256, 0, s>>>(nrp, elig, skip, n, o.maps, o.gshift, bc, nb);
    scan_inclusive(bc, SPMM_NT * nb, s, ar);
    k_sched_place<<<(unsigned)nb, 256, 0, s>>>(nrp, elig, skip, n, o.maps, o.gshift, bc, nb, rows);
    k_sched_totals<<<1, 64, 0, s>>>(bc, nb, dtot);
    read_back(tot, dtot, sizeof(tot), s);
  }
  int64_t prev = 0, blocks = 0;
  for (int ty = 0; ty < SPMM_NT; ty++) {
    const int G = 4 << (ty < 4 ? ty : ty - 4);
    const int64_t cnt = tot[ty] - prev;
    S.row_off[ty] = prev;
    S.blk_off[ty] = blocks;
    blocks += ((cnt + (SPMM_BS / G) - 1) / (SPMM_BS / G) + 7) & ~(int64_t)7;
    prev = tot[ty];
  }
  S.row_off[SPMM_NT] = prev;
  S.blk_off[SPMM_NT] = blocks;
  S.rows = rows;
  S.xcd_split = o.xcd_split;
  S.unroll = o.unroll;
  S.bmap = nullptr;
  if (o.xcd_split == XCD_MERGED && blocks) {
    if (blocks >= (int64_t(1) << 27)) throw Error(EMIN_ERR_CAPACITY, "masked product: too many blocks");
    int32_t* bmap = ar.alloc<int32_t>(blocks);
    MergeArgs A;
    A.rows = rows;
    for (int t = 0; t <= SPMM_NT; t++) {
      A.row_off[t] = S.row_off[t];
      A.blk_off[t] = S.blk_off[t];
    }
    k_sched_merge<<<nblocks(blocks, 256), 256, 0, s>>>(A, bmap);
    S.bmap = bmap;
  }
}

// ---------------------------------------------------------------------------
// Autotuner of the masked product's schedule.  The candidates (maps on/off,
// lanes per row tight or doubled, XCD split by class or contiguous) are timed
// on the pattern itself (median of three products, HIP events); the winner is
// kept in a process-wide table keyed by the shape of the problem (row count,
// mean row lengths of M and of the pattern, longest pattern row, bucketed),
// so later patterns of the same shape reuse it without timing.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::map<std::array<int64_t, 4>, SchedOpts> g_tune;
int64_t g_tune_stats[3] = {0, 0, 0};   // timed, reused, candidates timed

std::array<int64_t, 4> shape_key(const EminWork& w, const Csr& M) {
  auto lg = [](double v) { return (int64_t)std::llround(2.0 * std::log2(v > 1.0 ? v : 1.0)); };
  return {lg((double)w.n), lg(w.n ? (double)M.nnz / w.n : 1.0),
          lg(w.n ? (double)w.nnz / w.n : 1.0), (int64_t)w.smax};
}
}  // namespace

void EminWork::make_bins(const Csr& M, const int64_t* nrp, const int32_t* ncol, hipStream_t s,
                         Arena& ar, bool tune, bool stage, const double* xyz,
                         const int32_t* xmap, int dim) {
  nnzm = M.nnz;
  if (n) HIP_OK(hipMemsetAsync(rowdot, 0, sizeof(double) * n, s));   // empty rows stay 0
  nplanes = smax <= 8 ? 1 : (smax <= 16 ? 2 : 4);
  kofs = ar.alloc<int32_t>(M.nnz);
  nib = ar.alloc<uint32_t>((size_t)M.nnz * nplanes);
  uint8_t* elig = ar.alloc<uint8_t>(n);
  if (n) {
    const double avg = (double)M.nnz / (double)n;
    int g = 4;
    while (g < 64 && g < avg) g <<= 1;
    switch (g) {
      case 4: k_spmm_maps<4><<<nblocks(n, 64), 256, 0, s>>>(M.rowptr, M.col, nrp, ncol, n, nnzm, nplanes, kofs, nib, elig); break;
      case 8: k_spmm_maps<8><<<nblocks(n, 32), 256, 0, s>>>(M.rowptr, M.col, nrp, ncol, n, nnzm, nplanes, kofs, nib, elig); break;
      case 16: k_spmm_maps<16><<<nblocks(n, 16), 256, 0, s>>>(M.rowptr, M.col, nrp, ncol, n, nnzm, nplanes, kofs, nib, elig); break;
      case 32: k_spmm_maps<32><<<nblocks(n, 8), 256, 0, s>>>(M.rowptr, M.col, nrp, ncol, n, nnzm, nplanes, kofs, nib, elig); break;
      default: k_spmm_maps<64><<<nblocks(n, 4), 256, 0, s>>>(M.rowptr, M.col, nrp, ncol, n, nnzm, nplanes, kofs, nib, elig); break;
    }
  }
  tuned = 0;
  opts = SchedOpts{};
  opts.stage = stage;   // the tiled product is chosen by the caller
  this->stage = StagePlan{};
  if (n && stage) stage_plan(*this, M, nrp, elig, xyz, xmap, dim, s, ar);
  if (!tune || n == 0) {
    build_sched(*this, nrp, elig, opts, sched, s, ar);
    return;
  }
  const auto key = shape_key(*this, M);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      g_tune_stats[1]++;
      opts = it->second;
      opts.stage = stage;
      tuned = 2;
      build_sched(*this, nrp, elig, opts, sched, s, ar);
      return;
    }
  }
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float best = 1e30f;
  SchedOpts bo{};
  SpmmSched bs{};
  int ncand = 0;
  for (int maps = 1; maps >= 0; maps--)
    for (int gshift = 0; gshift <= 1; gshift++)
      for (int xs = XCD_MERGED; xs >= XCD_CONTIGUOUS; xs--)
        for (int un = 4; un <= (maps ? 16 : 4); un += 12) {
        const SchedOpts o{maps != 0, gshift, xs, stage, un};
        SpmmSched S{};
        build_sched(*this, nrp, elig, o, S, s, ar);
        const SpmmSched keep = sched;
        sched = S;
        float t[3];
        for (int r = 0; r < 3; r++) {
          HIP_OK(hipEventRecord(e0, s));
          masked_spmm(*this, M, nrp, ncol, Z, Q, nullptr, part, nullptr, s);
          HIP_OK(hipEventRecord(e1, s));
          HIP_OK(hipEventSynchronize(e1));
          HIP_OK(hipEventElapsedTime(&t[r], e0, e1));
        }
        sched = keep;
        std::sort(t, t + 3);
        ncand++;
        // the default schedule (timed first) is kept unless another beats it
        // by 5 %: a product timed alone only roughly predicts one running
        // beside other work, as in batches
        const SchedOpts d{};
        const bool is_def = o.maps == d.maps && o.gshift == d.gshift &&
                            o.xcd_split == d.xcd_split && o.unroll == d.unroll;
        const float score = is_def ? t[1] : t[1] / 0.95f;
        if (score < best) {
          best = score;
          bo = o;
          bs = S;
        }
      }
  HIP_OK(hipEventDestroy(e0));
  HIP_OK(hipEventDestroy(e1));
  sched = bs;
  opts = bo;
  tuned = 1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = bo;
  g_tune_stats[0]++;
  g_tune_stats[2] += ncand;
}

int32_t EminWork::sched_code() const {
  return (int32_t)((opts.maps ? 1 : 0) | (opts.gshift ? 2 : 0) |
                   (opts.xcd_split == XCD_BY_CLASS ? 4 : 0) |
                   (opts.xcd_split == XCD_MERGED ? 8 : 0) | (tuned << 4) |
                   ((opts.stage && stage.ntile) ? 64 : 0) | (opts.unroll >= 16 ? 128 : 0));
}

void autotune_stats(int64_t* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  out[0] = g_tune_stats[0];
  out[1] = g_tune_stats[1];
  out[2] = g_tune_stats[2];
  out[3] = (int64_t)g_tune.size();
}

void autotune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_stats[0] = g_tune_stats[1] = g_tune_stats[2] = 0;
}

// (when the product is timed, the launch itself records the events at the
// kernel's start and end, so the time excludes the gaps between launches)
template <class TM, class TX, class TY>
static void spmm_any(const EminWork& w, const Csr& M, const TM* mval, const int64_t* nrp,
                     const int32_t* ncol, const TX* X, TY* Y, const double* D, double bytes,
                     hipStream_t s) {
  // rows of staged tiles, then the rest: one timed interval from the first
  // launch's start to the last one's end
  const bool tiled = w.opts.stage && w.stage.ntile;
  const int64_t nb = w.sched.blk_off[SPMM_NT];
  if (!tiled && nb == 0) return;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = prof::begin_launch(s, EMIN_PROF_SPMM, bytes, 0.0, &e0, &e1);
  if (tiled)
    spmm_stage<TM, TX, TY>(w, M.rowptr, mval, nrp, X, Y, D, s, timed ? e0 : nullptr,
                           (timed && nb == 0) ? e1 : nullptr);
  if (nb == 0) return;
  if (timed) {
    hipExtLaunchKernelGGL(k_spmm<TM, TX, TY>, dim3((unsigned)nb), dim3(SPMM_BS), 0, s,
                          tiled ? nullptr : e0, e1, 0, w.sched, (const int64_t*)M.rowptr,
                          (const int32_t*)M.col, mval, (const int32_t*)w.kofs,
                          (const uint32_t*)w.nib, w.nnzm, nrp, ncol, X, Y, D, w.rowdot);
    HIP_OK(hipGetLastError());
  } else {
    k_spmm<TM, TX, TY><<<(unsigned)nb, SPMM_BS, 0, s>>>(w.sched, M.rowptr, M.col, mval, w.kofs,
                                                     w.nib, w.nnzm, nrp, ncol, X, Y, D, w.rowdot);
  }
}

// The values the finaliser sums for <D, Y> (rows with an empty pattern keep
// rowdot = 0): up to 16K rows the per-row values themselves, above that the
// block sums of k_rowsum.  The choice depends on n only, so every schedule of
// the product gives the same scalar.
constexpr int64_t ROWDOT_DIRECT = 16384;
static int64_t rowdot_partials(const EminWork& w, double* part, const double** src,
                               hipStream_t s) {
  if (w.n <= ROWDOT_DIRECT) {
    *src = w.rowdot;
    return w.n;
  }
  const int64_t nb = (int64_t)nblocks(w.n, 1024);
  k_rowsum<<<(unsigned)nb, 256, 0, s>>>(w.rowdot, w.n, part);
  *src = part;
  return nb;
}

// algorithmic bytes of one masked product: M (col + val) and row pointers,
// the pattern's columns, X read once and Y written once
static double spmm_bytes(const EminWork& w, const Csr& M, bool mixed) {
  const double vb = mixed ? 4.0 : 8.0;
  return (4.0 + vb) * (double)M.nnz + (4.0 + 2.0 * vb) * (double)w.nnz + 16.0 * (double)(w.n + 1);
}

int64_t masked_spmm(const EminWork& w, const Csr& M, const int64_t* nrp, const int32_t* ncol,
                    const double* X, double* Y, const double* D, double* part,
                    const double** dots, hipStream_t s) {
  spmm_any<double, double, double>(w, M, M.val, nrp, ncol, X, Y, D, spmm_bytes(w, M, false), s);
  return D ? rowdot_partials(w, part, dots, s) : 0;
}

void run_emin(EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp, const int32_t* ncol,
              const int32_t* cid, const int32_t* clist, const double* W, double* P, int iters,
              bool energy, bool mixed, EminReportPtrs rp, hipStream_t s) {
  const int64_t n = w.n, nnz = w.nnz;
  if (n == 0) return;
  // W_c = W on the C points (without a C list, the caller has filled w.Wc)
  if (w.nc && clist) k_gather_modes<<<nblocks(w.nc, 256), 256, 0, s>>>(W, clist, w.nc, w.Wc);
  launch_emin_init(nrp, ncol, n, nnz, cid, W, w.Wc, w.G, P, rp.status, s);
  // E0 = <P0, mask(M P0)> and R = -Pi(mask(M P0))
  const double* dots = nullptr;
  int64_t np = masked_spmm(w, M, nrp, ncol, P, w.MP, P, w.part, &dots, s);
  k_finalize<<<1, 1024, 0, s>>>(dots, (int)np, w.sc, FIN_E0, 0, rp.energy, nullptr, nullptr,
                                nullptr, nullptr);
  const int64_t nbr = init_r(w, nrp, ncol, cid, s);
  k_finalize<<<1, 1024, 0, s>>>(w.part, (int)nbr, w.sc, FIN_RHO0, 0, nullptr, rp.rho, nullptr,
                                nullptr, nullptr);
  if (mixed) k_to_float<<<nblocks(nnz, 256), 256, 0, s>>>(w.Z, w.Zf, nnz);
  for (int it = 0; it < iters; it++) {
    if (mixed) {
      spmm_any<float, float, float>(w, M, Mf, nrp, ncol, w.Zf, w.Qf, w.Z, spmm_bytes(w, M, true),
                                    s);
      np = rowdot_partials(w, w.part, &dots, s);
    } else {
      np = masked_spmm(w, M, nrp, ncol, w.Z, w.Q, w.Z, w.part, &dots, s);
    }
    k_finalize<<<1, 1024, 0, s>>>(dots, (int)np, w.sc, FIN_GAMMA, it, nullptr, nullptr,
                                  rp.gamma, rp.its, rp.status);
    int64_t nbu = 0;
    {
    const double ub = (mixed ? 40.0 : 44.0) * (double)nnz + 20.0 * (double)n +
                      (energy ? 16.0 * (double)nnz : 0.0);
    prof::Scope pu(s, EMIN_PROF_UPDATE, ub);
    nbu = cg_update(w, nrp, ncol, cid, P, energy, mixed, s);
    }
    k_finalize<<<1, 1024, 0, s>>>(w.part, (int)nbu, w.sc, FIN_RHO, it, nullptr, rp.rho, nullptr,
                                  nullptr, nullptr);
    if (energy)
      k_finalize<<<1, 1024, 0, s>>>(w.part_e, (int)nbu, w.sc, FIN_E, it, rp.energy, nullptr,
                                    nullptr, nullptr, nullptr);
    k_zupd<<<nblocks(nnz, 256), 256, 0, s>>>(w.R, w.Z, mixed ? w.Zf : nullptr, nnz, w.sc);
  }
}

void gather_modes(const double* W, const int32_t* clist, int64_t nc, double* Wc, hipStream_t s) {
  if (nc) k_gather_modes<<<nblocks(nc, 256), 256, 0, s>>>(W, clist, nc, Wc);
}

void emin_init(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz, const int32_t* cid,
               const double* W, const double* Wc, double* G, double* P, int32_t* status,
               hipStream_t s) {
  if (n) launch_emin_init(rp, col, n, nnz, cid, W, Wc, G, P, status, s);
}

__global__ void k_to_double(const float* a, double* b, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (double)a[e];
}

void masked_product(const EminWork& w, const Csr& M, const float* Mf, const int64_t* nrp,
                    const int32_t* ncol, const double* X, double* Y, bool mixed, hipStream_t s) {
  if (!mixed) {
    spmm_any<double, double, double>(w, M, M.val, nrp, ncol, X, Y, nullptr,
                                     spmm_bytes(w, M, false), s);
    return;
  }
  if (w.nnz) k_to_float<<<nblocks(w.nnz, 256), 256, 0, s>>>(X, w.Zf, w.nnz);
  spmm_any<float, float, float>(w, M, Mf, nrp, ncol, w.Zf, w.Qf, nullptr, spmm_bytes(w, M, true),
                                s);
  if (w.nnz) k_to_double<<<nblocks(w.nnz, 256), 256, 0, s>>>(w.Qf, Y, w.nnz);
}

void default_modes(const uint8_t* dir, int64_t n, double* W, hipStream_t s) {
  if (n) k_default_modes<<<nblocks(n, 256), 256, 0, s>>>(dir, n, W);
}

void to_float(const double* a, float* b, int64_t n, hipStream_t s) {
  if (n) k_to_float<<<nblocks(n, 256), 256, 0, s>>>(a, b, n);
}

}  // namespace emin
