// Alg. 3 (find_coarse_pressures) with update_heuristics and
// find_extra_dist3_Cpoints, as persistent single-workgroup kernels.
//
// Alg. 3 is a sequential greedy: every step picks the candidate with the
// smallest heuristic h1, and that choice changes the candidates and keys
// within graph distance 4.  One workgroup runs the loop; each step's BFS,
// state update and argmin are spread over its 1024 lanes.  The argmin is
// kept in LDS as per-block minima over fixed blocks of vertices, and only
// blocks touched by the step are recomputed.  The floating-point work that
// decides integers (distances, 1/d sums, h1 = cnt/rs, the extra-point tests)
// uses the same operations in the same order as the definition, with
// contraction disabled, so the result is bit-identical to it.
#include "coarsen.h"
#include "prof.h"

namespace emin {

constexpr int A3_BS = 1024;
constexpr int A3_WAVES = A3_BS / 64;

__device__ __forceinline__ double euclid(const double* x, int dim, int64_t a, int64_t b) {
  double s = 0.0;
  for (int d = 0; d < dim; d++) {
    const double t = x[a * dim + d] - x[b * dim + d];
    s = s + t * t;
  }
  return sqrt(s);
}

__device__ __forceinline__ bool lex_less(double ka, int32_t ia, double kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Every vertex's distance-4 ball, listed in BFS level order as
// (vertex | distance << 29), computed once in parallel (one wave per vertex,
// LDS hash set).  Each greedy step then reads the ball of its new C point in
// one coalesced sweep instead of walking the graph.
constexpr int BW = 4;          // waves per block
constexpr int BHASH = 4096;    // LDS hash slots per wave
constexpr int BLIST = 2048;    // ball capacity per wave
constexpr int DSHIFT = 29;
constexpr int32_t VMASK = (1 << DSHIFT) - 1;

__device__ __forceinline__ uint32_t bhash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(64 * BW) void k_balls(const int64_t* grp, const int32_t* gcol,
                                                   int64_t n, int depth, int32_t* bsize,
                                                   int32_t* b3, int32_t* balls, int bmax,
                                                   int* err) {
  extern __shared__ int32_t lds_b[];
  __shared__ int nb_all[BW];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t v0 = (int64_t)blockIdx.x * BW + w;
  if (v0 >= n) return;
  int32_t* hs = lds_b + w * (BHASH + BLIST);
  int32_t* ball = hs + BHASH;
  for (int t = lane; t < BHASH; t += 64) hs[t] = -1;
  if (lane == 0) {
    ball[0] = (int32_t)v0;
    hs[bhash((uint32_t)v0) & (BHASH - 1)] = (int32_t)v0;
    nb_all[w] = 1;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int ls = 0, le = 1;
  int ends[5] = {1, 1, 1, 1, 1};
  bool bad = false;
  for (int L = 0; L < depth; L++) {
    for (int f = ls + lane; f < le; f += 64) {
      const int32_t v = ball[f];
      for (int64_t e = grp[v]; e < grp[v + 1]; e++) {
        const int32_t u = gcol[e];
        if (u == v) continue;
        uint32_t h = bhash((uint32_t)u) & (BHASH - 1);
        int probes = 0;
        while (true) {
          const int32_t old = atomicCAS(&hs[h], -1, u);
          if (old == -1) {
            const int p = atomicAdd(&nb_all[w], 1);
            if (p < BLIST) ball[p] = u; else bad = true;
            break;
          }
          if (old == u) break;
          h = (h + 1) & (BHASH - 1);
          if (++probes >= BHASH / 2) { bad = true; break; }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    ls = le;
    le = min(nb_all[w], BLIST);
    ends[L + 1] = le;
  }
  for (int L = depth + 1; L < 5; L++) ends[L] = le;
  if (bad || le > bmax) {
    if (lane == 0) atomicOr(err, DERR_CAPACITY);
    return;
  }
  if (lane == 0) {
    bsize[v0] = le;
    b3[v0] = ends[3];
  }
  if (!balls) return;
  int32_t* out = balls + v0 * (int64_t)bmax;
  for (int t = lane; t < le; t += 64) {
    int d = 0;
    while (d < 4 && t >= ends[d]) d++;
    out[t] = (int32_t)((uint32_t)ball[t] | ((uint32_t)d << DSHIFT));
  }
}

// Distance-4 balls with a visited bitmap over the index window of the ball
// (8 bw + 1 bits) instead of a hash set: one atomic OR per edge, no probing,
// little LDS, so many waves per CU.  One wave per vertex, BFS level by level;
// entries (vertex | distance << 29) in level order, at most lcap per ball
// (a longer ball sets the overflow flag and leaves its row unwritten).
constexpr int BWIN_W = 4;   // waves per block

__global__ __launch_bounds__(64 * BWIN_W) void k_balls_win(const int64_t* grp,
                                                           const int32_t* gcol, int64_t n,
                                                           const int32_t* verts, int64_t bw,
                                                           int nwords, int lcap, int32_t* bsize,
                                                           int32_t* b3, int32_t* balls,
                                                           int64_t stride, int* flags) {
  extern __shared__ uint32_t lds_w[];
  __shared__ int cnt[BWIN_W];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * BWIN_W + w;
  if (r >= n) return;   // whole wave; the block never synchronises
  const int64_t v0 = verts ? verts[r] : r;
  uint32_t* bits = lds_w + (size_t)w * (nwords + lcap);
  int32_t* list = reinterpret_cast<int32_t*>(bits + nwords);
  const int64_t lo = v0 - 4 * bw > 0 ? v0 - 4 * bw : 0;
  for (int t = lane; t < nwords; t += 64) bits[t] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane == 0) {
    const int64_t o = v0 - lo;
    bits[o >> 5] |= 1u << (o & 31);
    list[0] = (int32_t)v0;
    cnt[w] = 1;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int ls = 0, le = 1;
  int ends[5] = {1, 1, 1, 1, 1};
  for (int L = 0; L < 4; L++) {
    for (int f = ls + lane; f < le; f += 64) {
      const int32_t v = list[f];
      const int64_t ea = grp[v], eb = grp[v + 1];
      for (int64_t e = ea; e < eb; e += 4) {
        int32_t u[4];
#pragma unroll
        for (int q = 0; q < 4; q++) u[q] = e + q < eb ? gcol[e + q] : v;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          if (u[q] == v) continue;
          const int64_t o = (int64_t)u[q] - lo;
          const uint32_t bit = 1u << (o & 31);
          if ((atomicOr(&bits[o >> 5], bit) & bit) == 0u) {
            const int p = atomicAdd(&cnt[w], 1);
            if (p < lcap) list[p] = u[q];
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int c = cnt[w];
    if (c > lcap) {
      if (lane == 0) atomicOr(flags, 1);
      return;
    }
    ls = le;
    le = c;
    ends[L + 1] = le;
  }
  if (lane == 0) {
    bsize[v0] = le;
    b3[v0] = ends[3];
    // a relaxed read first: most balls are not larger than one already seen,
    // and same-address atomics from every vertex would serialise
    if (le > __hip_atomic_load(flags + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(flags + 1, le);
  }
  if (!balls) return;
  int32_t* out = balls + v0 * stride;
  for (int t = lane; t < le; t += 64) {
    int d = 0;
    while (d < 4 && t >= ends[d]) d++;
    out[t] = (int32_t)((uint32_t)list[t] | ((uint32_t)d << DSHIFT));
  }
}

__global__ void k_sample_verts(int64_t n, int32_t m, int32_t* verts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) verts[i] = (int32_t)(((int64_t)i * n) / m);
}

__device__ __forceinline__ void s_append(const CoarsenArgs& D, int32_t v, int32_t c, int d,
                                         int* err_sh) {
  const int sl = D.s_cnt[v];
  if (sl < D.scap) {
    D.s_c[(int64_t)v * D.scap + sl] = c;
    D.s_d[(int64_t)v * D.scap + sl] = (uint8_t)d;
    D.s_cnt[v] = sl + 1;
  } else {
    atomicOr(err_sh, DERR_CAPACITY);
  }
}

__device__ __forceinline__ void mark_dirty(int b, uint32_t* dbits, int32_t* dlist, int dcap,
                                           int* dn, int* dall, int32_t* bslot = nullptr) {
  const uint32_t bit = 1u << (b & 31);
  if ((atomicOr(&dbits[b >> 5], bit) & bit) == 0) {
    const int p = atomicAdd(dn, 1);
    if (p < dcap) dlist[p] = b;
    else *dall = 1;
    if (bslot) bslot[b] = p;
  }
}

// Alg. 3 keeps, for at most A3_OVL touched blocks of 64 vertices, an LDS
// overlay of the keys the step has just written, so the refresh can combine
// them with keys loaded before the update (those of untouched vertices are
// unchanged) instead of reloading the block after its stores.
constexpr int A3_OVL = 64;

__global__ void k_fill_inf(double* a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = __builtin_inf();
}

// One greedy step costs a few dependent memory round trips, so the loop is
// arranged to keep that chain short: the new C point's ball is fetched
// together with its size, every per-vertex field a ball entry needs is loaded
// before any is stored, and the heuristic key of each candidate (h1 = cnt/rs,
// +inf for a non-candidate) is kept in its own array so that refreshing a
// block's minimum is a single coalesced read.
// per-thread copy of one ball entry's vertex state (set only in waves that
// hold entries, and read only there)
struct A3Entry {
  int32_t v, d, s, c, sl;
  double r, x0, x1, x2;
};

template <bool OVL>
__global__ __launch_bounds__(A3_BS) void k_alg3(CoarsenArgs D) {
  extern __shared__ unsigned char lds_raw[];
  double* bkey = reinterpret_cast<double*>(lds_raw);
  int32_t* bidx = reinterpret_cast<int32_t*>(bkey + D.nblk);
  // dirty-block sets are double-buffered by step parity, so a set can be
  // cleared right after its refresh
  const int nw = (D.nblk + 31) / 32;
  uint32_t* dbits0 = reinterpret_cast<uint32_t*>(bidx + D.nblk);
  int32_t* dlist0 = reinterpret_cast<int32_t*>(dbits0 + 2 * nw);
  // overlay (64-vertex blocks only): slot of each touched block, and keys
  int32_t* bslot = dlist0 + 2 * D.dcap;
  const size_t ovl_off =
      ((size_t)D.nblk * 12 + (size_t)nw * 8 + (size_t)D.dcap * 8 + ((size_t)D.nblk + 1) * 4 + 7) &
      ~(size_t)7;
  double* ovl = reinterpret_cast<double*>(lds_raw + ovl_off);
  constexpr bool ovl_ok = OVL;   // 64-vertex blocks
  __shared__ int err_sh, nc_sh, cursor_sh, found_sh;
  __shared__ int dn_sh[2], dall_sh[2];
  __shared__ double wkey[A3_WAVES];
  __shared__ int32_t widx[A3_WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double INF = __builtin_inf();
  const int64_t n = D.n;
  const int dim = D.dim;

  for (int b = tid; b < D.nblk; b += A3_BS) { bkey[b] = INF; bidx[b] = INT32_MAX; }
  for (int b = tid; b < 2 * nw; b += A3_BS) dbits0[b] = 0u;
  if (ovl_ok)
    for (int t = tid; t < A3_OVL * 64; t += A3_BS) ovl[t] = -1.0;
  if (tid == 0) {
    err_sh = 0; nc_sh = 0; cursor_sh = 0;
    dn_sh[0] = dn_sh[1] = 0;
    dall_sh[0] = dall_sh[1] = 0;
  }
  __syncthreads();
  int par = 0;

  int32_t k = n > 0 ? 0 : -1;   // Alg. 3's "arbitrary vertex": vertex 0
  while (k >= 0) {
    uint32_t* dbits = dbits0 + par * nw;
    int32_t* dlist = dlist0 + par * D.dcap;
    // (1) the ball of k (at most two entries per thread), dirty marks, and
    // the loads of every per-vertex field the entries need
    const int32_t* bl = D.balls + (int64_t)k * D.bstride;
    const int32_t ea = tid < D.bmax ? bl[tid] : 0;
    const int32_t eb = tid + A3_BS < D.bmax ? bl[tid + A3_BS] : 0;
    const int nb = D.bsize[k];
    const double* xkp = D.x + (int64_t)k * dim;
    const double xk0 = xkp[0], xk1 = xkp[1], xk2 = dim == 3 ? xkp[2] : 0.0;
    // (k's coordinates arrive with the ball: retiring them here keeps their
    // registers free of pending loads on every later path, where a wait for
    // them would be a wait for the whole in-order load counter)
    asm volatile("" ::"v"(ea), "v"(xk0), "v"(xk1), "v"(xk2) : "memory");
    const int nc0 = nc_sh;
    A3Entry E[2];
    const bool has[2] = {tid < nb, tid + A3_BS < nb};
    const bool wh[2] = {wave * 64 < nb, A3_BS + wave * 64 < nb};   // wave-uniform
    // (inside a wave that holds entries the loads are unconditional, from k
    // itself for a lane without one, so that no register merge waits for them)
#pragma unroll
    for (int q = 0; q < 2; q++) {
      if (!wh[q]) continue;
      const int32_t e = q ? eb : ea;
      A3Entry& x = E[q];
      x.v = has[q] ? (e & VMASK) : k;
      x.d = (int)((uint32_t)e >> DSHIFT);
      if (has[q])
        mark_dirty(x.v / D.vb, dbits, dlist, D.dcap, &dn_sh[par], &dall_sh[par],
                   ovl_ok ? bslot : nullptr);
      x.s = D.st[x.v];
      x.c = D.cnt[x.v];
      x.r = D.rs[x.v];
      x.sl = D.s_cnt[x.v];
      const double* xvp = D.x + (int64_t)x.v * dim;
      x.x0 = xvp[0];
      x.x1 = xvp[1];
      x.x2 = xvp[dim == 3 ? 2 : 1];
    }
    __syncthreads();
    // (2) while those loads are in flight: the pre-update keys of the touched
    // blocks (overlay mode), and the minimum over the blocks this step leaves
    // untouched (their stored minima are current)
    const bool all = dall_sh[par] != 0;
    const int todo = all ? D.nblk : dn_sh[par];
    const bool use_ovl = ovl_ok && !all && todo <= A3_OVL;   // uniform
    // (issued unconditionally, from clamped addresses, so that the number of
    // loads in flight is the same on every path and later waits stay exact)
    double oldk[A3_OVL / A3_WAVES];
    if (ovl_ok) {
#pragma unroll
      for (int i = 0; i < A3_OVL / A3_WAVES; i++) {
        const int t = wave + A3_WAVES * i;
        const int64_t v = (int64_t)dlist[t < todo ? t : 0] * 64 + lane;
        const double h = D.hkey[v < n ? v : n - 1];
        oldk[i] = (use_ovl && t < todo && v < n) ? h : INF;
      }
    }
    double ck = INF;
    int32_t ci = INT32_MAX;
    for (int b = tid; b < D.nblk; b += A3_BS)
      if (!((dbits[b >> 5] >> (b & 31)) & 1u) && lex_less(bkey[b], bidx[b], ck, ci)) {
        ck = bkey[b];
        ci = bidx[b];
      }
    wave_argmin(ck, ci);
    // the loaded fields are first used here (an empty asm that "modifies"
    // them keeps the compiler from consuming them before the scan)
#pragma unroll
    for (int q = 0; q < 2; q++)
      if (wh[q])
        asm volatile("" : "+v"(E[q].s), "+v"(E[q].c), "+v"(E[q].r), "+v"(E[q].sl),
                     "+v"(E[q].x0), "+v"(E[q].x1), "+v"(E[q].x2));
    // (3) S_j += {k} for dist <= 3; C/F/Cand update; update_heuristics
#pragma unroll
    for (int q = 0; q < 2; q++) {
      if (!has[q]) continue;
      const A3Entry& x = E[q];
      if (x.d <= 3) {   // S_v += {k}; S_k holds k itself
        if (x.sl < D.scap) {
          D.s_c[(int64_t)x.v * D.scap + x.sl] = k;
          D.s_d[(int64_t)x.v * D.scap + x.sl] = (uint8_t)x.d;
          D.s_cnt[x.v] = x.sl + 1;
        } else {
          atomicOr(&err_sh, DERR_CAPACITY);
        }
      }
      if (x.d == 0) {
        D.st[x.v] = ST_C;
        D.hkey[x.v] = INF;
        D.order[nc0] = x.v;
        if (use_ovl) ovl[bslot[x.v >> 6] * 64 + (x.v & 63)] = INF;
      } else {
        // |x_v - x_k| summed in coordinate order, as in the definition
        const double t0 = x.x0 - xk0, t1 = x.x1 - xk1, t2 = (dim == 3 ? x.x2 : 0.0) - xk2;
        double ss = 0.0;
        ss = ss + t0 * t0;
        ss = ss + t1 * t1;
        if (dim == 3) ss = ss + t2 * t2;
        const double r1 = x.r + 1.0 / sqrt(ss);
        const int32_t c1 = x.c + 1;
        int32_t s1 = x.s;
        if (x.d <= 3 && (x.s == ST_U || x.s == ST_CAND)) s1 = ST_F;
        if (x.d == 4 && x.s == ST_U) s1 = ST_CAND;
        if (s1 != x.s) D.st[x.v] = (uint8_t)s1;
        D.cnt[x.v] = c1;
        D.rs[x.v] = r1;
        const double nk = s1 == ST_CAND ? (double)c1 / r1 : INF;
        if (s1 == ST_CAND || x.s == ST_CAND) D.hkey[x.v] = nk;
        if (use_ovl) ovl[bslot[x.v >> 6] * 64 + (x.v & 63)] = nk;
      }
    }
    __syncthreads();
    if (tid == 0) nc_sh = nc0 + 1;
    // (4) new minima of the touched blocks, folded into the wave's minimum
    if (use_ovl) {
#pragma unroll
      for (int i = 0; i < A3_OVL / A3_WAVES; i++) {
        const int t = wave + A3_WAVES * i;
        if (t >= todo) break;   // wave-uniform
        const int b = dlist[t];
        const double o = ovl[t * 64 + lane];
        ovl[t * 64 + lane] = -1.0;
        const double h1 = o != -1.0 ? o : oldk[i];
        double key = INF;
        int32_t idx = INT32_MAX;
        if (h1 < INF) { key = h1; idx = b * 64 + lane; }
        wave_argmin(key, idx);
        if (lane == 0) { bkey[b] = key; bidx[b] = idx; }
        if (lex_less(key, idx, ck, ci)) { ck = key; ci = idx; }
      }
    } else for (int t = wave; t < todo; t += A3_WAVES) {
      const int b = all ? t : dlist[t];
      double key = INF;
      int32_t idx = INT32_MAX;
      if (D.vb == 64) {
        const int64_t v = (int64_t)b * 64 + lane;
        const double h1 = v < n ? D.hkey[v] : INF;
        if (h1 < INF) { key = h1; idx = (int32_t)v; }
      } else for (int u0 = 0; u0 < D.vb; u0 += 256) {
        double h[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int64_t v = (int64_t)b * D.vb + u0 + lane + 64 * j;
          h[j] = (u0 + lane + 64 * j < D.vb && v < n) ? D.hkey[v] : INF;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int32_t v = (int32_t)((int64_t)b * D.vb + u0 + lane + 64 * j);
          if (h[j] < INF && lex_less(h[j], v, key, idx)) { key = h[j]; idx = v; }
        }
      }
      wave_argmin(key, idx);
      if (lane == 0) { bkey[b] = key; bidx[b] = idx; }
      if (lex_less(key, idx, ck, ci)) { ck = key; ci = idx; }
    }
    // retire every pre-update key load on both refresh paths (they were
    // issued long before): a load left pending here would make a later
    // register reuse wait for the whole in-order load counter
    if (ovl_ok) {
#pragma unroll
      for (int i = 0; i < A3_OVL / A3_WAVES; i++) asm volatile("" ::"v"(oldk[i]));
    }
    if (lane == 0) { wkey[wave] = ck; widx[wave] = ci; }
    __syncthreads();
    // this step's dirty set is next used two steps on, after three barriers
    for (int b = tid; b < nw; b += A3_BS) dbits[b] = 0u;
    if (tid == 0) { dn_sh[par] = 0; dall_sh[par] = 0; }
    par ^= 1;
    // (5) next k = argmin over Cand of (h1, index): every wave reduces the
    // wave minima itself
    double key = lane < A3_WAVES ? wkey[lane] : INF;
    int32_t idx = lane < A3_WAVES ? widx[lane] : INT32_MAX;
    wave_argmin(key, idx);
    // an error ends the loop for every thread at the same point
    if (err_sh) break;
    k = idx;
    if (k == INT32_MAX) {
      // Cand is empty: the smallest-index unmarked vertex (the cursor only
      // moves forward: marks are permanent)
      if (tid == 0) found_sh = INT32_MAX;
      __syncthreads();
      for (int64_t base = cursor_sh; base < n; base += A3_BS) {
        const int64_t v = base + tid;
        if (v < n && D.st[v] == ST_U) atomicMin(&found_sh, (int)v);
        __syncthreads();
        const int f = found_sh;
        __syncthreads();
        if (f != INT32_MAX) break;
      }
      k = found_sh == INT32_MAX ? -1 : found_sh;
      __syncthreads();
      if (tid == 0 && k >= 0) cursor_sh = k;
    }
  }
  __syncthreads();
  if (tid == 0) {
    D.meta[0] = nc_sh;
    D.meta[1] = nc_sh;
    D.meta[2] |= err_sh;
  }
}

// mean Euclidean length of each vertex's graph edges
__global__ void k_ebar(CoarsenArgs D, double* ebar) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.n) return;
  double s = 0.0;
  int64_t deg = 0;
  for (int64_t e = D.grp[j]; e < D.grp[j + 1]; e++) {
    const int32_t w = D.gcol[e];
    if (w == j) continue;
    s = s + euclid(D.x, D.dim, j, w);
    deg++;
  }
  ebar[j] = deg ? s / (double)deg : 0.0;
}

// find_extra_dist3_Cpoints predicate of pass 1 / pass 2 with the current S
__device__ bool extra_pred(const CoarsenArgs& D, const double* ebar, int pass, int64_t j) {
  if (D.st[j] != ST_F) return false;
  const int sc = D.s_cnt[j];
  const int32_t* c = D.s_c + j * D.scap;
  const uint8_t* dd = D.s_d + j * D.scap;
  const double eb = ebar[j];
  if (pass == 1) {
    if (sc != 1) return false;
    return dd[0] == 3 && euclid(D.x, D.dim, j, c[0]) > 2.5 * eb;
  }
  if (sc != 2 || dd[0] != 3 || dd[1] != 3) return false;
  const int64_t a = c[0], b = c[1];
  const double ea = euclid(D.x, D.dim, j, a), ebb = euclid(D.x, D.dim, j, b);
  if (!(0.5 * (ea + ebb) > 2.5 * eb)) return false;
  const int dim = D.dim;
  const double* x = D.x;
  double num = 0.0, den = 0.0;
  for (int d = 0; d < dim; d++) {
    const double ab = x[b * dim + d] - x[a * dim + d];
    const double aj = x[j * dim + d] - x[a * dim + d];
    num = num + aj * ab;
    den = den + ab * ab;
  }
  double t = den > 0.0 ? num / den : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double s = 0.0;
  for (int d = 0; d < dim; d++) {
    const double ab = x[b * dim + d] - x[a * dim + d];
    const double q = x[a * dim + d] + t * ab;
    const double r = x[j * dim + d] - q;
    s = s + r * r;
  }
  return sqrt(s) > 1.0 * eb;
}

// Both passes in ascending order.  The state changes only when a vertex is
// converted, so the next conversion is the smallest vertex at or after the
// cursor whose predicate holds now; the workgroup finds it 1024 at a time.
__global__ __launch_bounds__(A3_BS) void k_extras(CoarsenArgs D, const double* ebar) {
  __shared__ int err_sh, found_sh, nc_sh;
  const int tid = threadIdx.x;
  if (tid == 0) {
    err_sh = 0;
    nc_sh = D.meta[0];
  }
  __syncthreads();
  for (int pass = 1; pass <= 2; pass++) {
    int64_t cursor = 0;
    while (true) {
      if (tid == 0) found_sh = INT32_MAX;
      __syncthreads();
      for (int64_t base = cursor; base < D.n; base += A3_BS) {
        const int64_t v = base + tid;
        if (v < D.n && extra_pred(D, ebar, pass, v)) atomicMin(&found_sh, (int)v);
        __syncthreads();
        const int f = found_sh;
        __syncthreads();
        if (f != INT32_MAX) break;
      }
      const int j = found_sh;
      if (j == INT32_MAX) break;
      // j becomes C and joins the S set of every vertex within distance 3
      const int n3 = D.b3[j];
      const int32_t* bl = D.balls + (int64_t)j * D.bstride;
      for (int t = tid; t < n3; t += A3_BS) {
        const int32_t e = bl[t];
        s_append(D, e & VMASK, j, (int)((uint32_t)e >> DSHIFT), &err_sh);
      }
      if (tid == 0) {
        D.st[j] = ST_C;
        D.order[nc_sh] = j;
        nc_sh++;
      }
      __syncthreads();
      cursor = (int64_t)j + 1;
      if (err_sh) break;
    }
    __syncthreads();
    if (err_sh) break;
  }
  if (tid == 0) {
    D.meta[0] = nc_sh;
    D.meta[2] |= err_sh;
  }
}

// Given C^(p) (ascending fine indices, checked here) instead of Alg. 3:
// the C flags and the selection order.
__global__ void k_given_mark(CoarsenArgs D, const int32_t* cp, int64_t ncp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    D.meta[0] = (int32_t)ncp;
    D.meta[1] = (int32_t)ncp;
  }
  if (t >= ncp) return;
  const int32_t c = cp[t];
  if (c < 0 || c >= D.n || (t > 0 && cp[t - 1] >= c)) {
    atomicOr(D.meta + 2, DERR_PATTERN);
    return;
  }
  D.st[c] = ST_C;
  D.order[t] = c;
}

// S_v = the C points within graph distance 3 of v, read off v's ball (its
// entries at distance <= 3 are a prefix); a vertex not given as C is F.
__global__ void k_given_sets(CoarsenArgs D) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= D.n) return;
  if (D.st[v] != ST_C) D.st[v] = ST_F;
  const int32_t* ball = D.balls + v * D.bstride;
  const int m = D.b3[v];
  int k = 0;
  for (int t = 0; t < m; t++) {
    const int32_t e = ball[t];
    const int32_t u = e & ((1 << 29) - 1);
    if (D.st[u] != ST_C) continue;
    if (k < D.scap) {
      D.s_c[v * D.scap + k] = u;
      D.s_d[v * D.scap + k] = (uint8_t)((uint32_t)e >> 29);
    } else {
      atomicOr(D.meta + 2, DERR_CAPACITY);
    }
    k++;
  }
  D.s_cnt[v] = k < D.scap ? k : D.scap;
}

// sort every S list by fine index (distances follow)
__global__ void k_sort_s(CoarsenArgs D) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  int32_t* c = D.s_c + i * D.scap;
  uint8_t* d = D.s_d + i * D.scap;
  const int m = D.s_cnt[i];
  for (int p = 1; p < m; p++) {
    const int32_t cv = c[p];
    const uint8_t dv = d[p];
    int q = p;
    while (q > 0 && c[q - 1] > cv) {
      c[q] = c[q - 1];
      d[q] = d[q - 1];
      q--;
    }
    c[q] = cv;
    d[q] = dv;
  }
}

// ---------------------------------------------------------------------------
// patterns from the C/F split
// ---------------------------------------------------------------------------
__global__ void k_flags_c(const uint8_t* st, int64_t n, int64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = st[i] == ST_C;
}

__global__ void k_compact(const int64_t* incl, const uint8_t* st, int64_t n, int32_t* list,
                          int32_t* cid) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool c = st[i] == ST_C;
  const int32_t id = c ? (int32_t)(incl[i] - 1) : -1;
  cid[i] = id;
  if (c) list[id] = (int32_t)i;
}

// meta[0..2] (|C|, |C| of Alg. 3, error bits) and the sizes of N^(p) and S
__global__ void k_coarse_summary(const int32_t* meta, const int64_t* nn, const int64_t* sn,
                                 int64_t* out) {
  if (threadIdx.x == 0) {
    out[0] = meta[0];
    out[1] = meta[1];
    out[2] = meta[2];
    out[3] = *nn;
    out[4] = *sn;
  }
}

__global__ void k_p_counts(const uint8_t* st, const int32_t* s_cnt, int64_t n, int64_t* nrp,
                           int64_t* srp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  nrp[i + 1] = st[i] == ST_C ? 1 : s_cnt[i];
  srp[i + 1] = s_cnt[i];
}

__global__ void k_p_fill(CoarsenArgs D, const int32_t* cid, const int64_t* nrp, int32_t* ncol,
                         const int64_t* srp, int32_t* scol, uint8_t* sdist) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  const int m = D.s_cnt[i];
  for (int t = 0; t < m; t++) {
    scol[srp[i] + t] = D.s_c[i * D.scap + t];
    sdist[srp[i] + t] = D.s_d[i * D.scap + t];
  }
  if (D.st[i] == ST_C) {
    ncol[nrp[i]] = cid[i];
  } else {
    for (int t = 0; t < m; t++) ncol[nrp[i] + t] = cid[D.s_c[i * D.scap + t]];
  }
}

void coarsen_pressure(CoarsenArgs& D, CoarsenOut& out, hipStream_t s, Arena& ar, int lds_max,
                      const int32_t* cp_given, int64_t ncp,
                      const std::function<void()>& overlap) {
  const int64_t n = D.n;
  D.st = ar.alloc<uint8_t>(n);
  D.cnt = ar.alloc<int32_t>(n);
  D.rs = ar.alloc<double>(n);
  D.hkey = ar.alloc<double>(n);
  D.s_cnt = ar.alloc<int32_t>(n);
  D.s_c = ar.alloc<int32_t>((size_t)n * D.scap);
  D.s_d = ar.alloc<uint8_t>((size_t)n * D.scap);
  D.order = ar.alloc<int32_t>(n);
  D.meta = ar.alloc<int32_t>(4);
  HIP_OK(hipMemsetAsync(D.st, 0, n, s));
  HIP_OK(hipMemsetAsync(D.cnt, 0, sizeof(int32_t) * n, s));
  HIP_OK(hipMemsetAsync(D.rs, 0, sizeof(double) * n, s));
  if (n) k_fill_inf<<<nblocks(n, 256), 256, 0, s>>>(D.hkey, n);
  HIP_OK(hipMemsetAsync(D.s_cnt, 0, sizeof(int32_t) * n, s));
  HIP_OK(hipMemsetAsync(D.meta, 0, sizeof(int32_t) * 4, s));
  // distance-4 balls of every vertex
  int32_t* bsize = ar.alloc<int32_t>(n);
  int32_t* b3 = ar.alloc<int32_t>(n);
  int32_t* balls = nullptr;
  int64_t bmax = 1, stride = 1;
  bool done = false;
  if (n) {
    // windowed bitmap kernel when the index bandwidth keeps the window small:
    // ball sizes of a sample of vertices pick the row capacity, then one pass
    // fills every row (a ball above the capacity repeats the pass, larger)
    int* flags = ar.alloc<int>(2);
    const int64_t bw = index_bandwidth(D.grp, D.gcol, n, s, ar);
    const int64_t nwords = (8 * bw + 1 + 31) / 32;
    int lcap = BLIST;
    auto lds_for = [&](int cap) { return (size_t)BWIN_W * (nwords + cap) * sizeof(uint32_t); };
    if (lds_for(BLIST) <= (size_t)lds_max) {
      allow_lds((const void*)k_balls_win);
      const int32_t m = (int32_t)std::min<int64_t>(n, 512);
      int32_t* sv = ar.alloc<int32_t>(m);
      k_sample_verts<<<nblocks(m, 256), 256, 0, s>>>(n, m, sv);
      HIP_OK(hipMemsetAsync(flags, 0, 2 * sizeof(int), s));
      k_balls_win<<<nblocks(m, BWIN_W), 64 * BWIN_W, lds_for(BLIST), s>>>(
          D.grp, D.gcol, m, sv, bw, (int)nwords, BLIST, bsize, b3, nullptr, 0, flags);
      int fl[2];
      read_back(fl, flags, sizeof(fl), s);
      if (fl[0] == 0) {
        lcap = 64;
        while (lcap < BLIST && lcap < fl[1] + fl[1] / 4) lcap <<= 1;
        for (int attempt = 0; attempt < 2 && !done; attempt++) {
          stride = lcap;
          balls = ar.alloc<int32_t>((size_t)n * stride);
          HIP_OK(hipMemsetAsync(flags, 0, 2 * sizeof(int), s));
          k_balls_win<<<nblocks(n, BWIN_W), 64 * BWIN_W, lds_for(lcap), s>>>(
              D.grp, D.gcol, n, nullptr, bw, (int)nwords, lcap, bsize, b3, balls, stride, flags);
          read_back(fl, flags, sizeof(fl), s);
          if (fl[0] == 0) {
            done = true;
            bmax = fl[1];
          } else {
            lcap = BLIST;
          }
        }
      }
    }
  }
  if (n && !done) {
    // hash-set kernel: sizes first, then the lists
    const size_t blds = (size_t)BW * (BHASH + BLIST) * sizeof(int32_t);
    allow_lds((const void*)k_balls);
    k_balls<<<nblocks(n, BW), 64 * BW, blds, s>>>(D.grp, D.gcol, n, 4, bsize, b3, nullptr, BLIST,
                                                  D.meta + 2);
    if (d2h(D.meta + 2, s) & DERR_CAPACITY) throw Error(EMIN_ERR_CAPACITY, "alg3: ball capacity");
    bmax = max_row_len_i32(bsize, n, s, ar);
    stride = bmax;
    balls = ar.alloc<int32_t>((size_t)n * stride);
    k_balls<<<nblocks(n, BW), 64 * BW, blds, s>>>(D.grp, D.gcol, n, 4, bsize, b3, balls,
                                                  (int)stride, D.meta + 2);
  }
  if (!n) balls = ar.alloc<int32_t>(1);
  D.balls = balls;
  D.bsize = bsize;
  D.b3 = b3;
  D.bmax = (int)bmax;
  D.bstride = stride;
  // LDS layout: block keys | block idx | dirty bits | dirty list
  // argmin blocks: 64 vertices where balls are small (few blocks touched per
  // step), 256 where they are large; at most two blocks per thread
  D.dcap = 1024;
  D.vb = D.bmax <= 128 ? 64 : 256;
  while ((n + D.vb - 1) / D.vb > 2 * A3_BS) D.vb <<= 1;
  D.nblk = (int)((n + D.vb - 1) / D.vb);
  if (D.nblk < 1) D.nblk = 1;
  size_t lds = (size_t)D.nblk * 12 + 2 * (size_t)((D.nblk + 31) / 32) * 4 + 2 * (size_t)D.dcap * 4 +
               ((size_t)D.nblk + 1) * 4 + 8 + (D.vb == 64 ? (size_t)A3_OVL * 64 * 8 : 0);
  if (lds > (size_t)lds_max) throw Error(EMIN_ERR_CAPACITY, "alg3: LDS too small");
  const void* kfun = D.vb == 64 ? (const void*)k_alg3<true> : (const void*)k_alg3<false>;
  allow_lds(kfun);
  if (cp_given) {
    // C^(p) given: the flags, the order and the S sets from the balls
    k_given_mark<<<nblocks(ncp > 0 ? ncp : 1, 256), 256, 0, s>>>(D, cp_given, ncp);
    if (n) k_given_sets<<<nblocks(n, 256), 256, 0, s>>>(D);
    HIP_OK(hipGetLastError());
  } else {
  prof::Scope ps(s, EMIN_PROF_ALG3, 0.0);
  if (D.vb == 64) k_alg3<true><<<1, A3_BS, lds, s>>>(D);
  else k_alg3<false><<<1, A3_BS, lds, s>>>(D);
  HIP_OK(hipGetLastError());
  double* ebar = ar.alloc<double>(n);
  if (n) k_ebar<<<nblocks(n, 256), 256, 0, s>>>(D, ebar);
  k_extras<<<1, A3_BS, 0, s>>>(D, ebar);
  HIP_OK(hipGetLastError());
  }
  if (n) k_sort_s<<<nblocks(n, 256), 256, 0, s>>>(D);
  // coarse numbering (ascending fine index), C list, S CSR, N^(p); the
  // counts of Alg. 3, its error bits and the two pattern sizes in one
  // read-back
  int64_t* incl = ar.alloc<int64_t>(n + 1);
  if (n) k_flags_c<<<nblocks(n, 256), 256, 0, s>>>(D.st, n, incl);
  scan_inclusive(incl, n, s, ar);
  out.N.nrows = n;
  out.N.rowptr = ar.alloc<int64_t>(n + 1);
  out.S.nrows = n;
  out.S.ncols = n;
  out.S.rowptr = ar.alloc<int64_t>(n + 1);
  HIP_OK(hipMemsetAsync(out.N.rowptr, 0, sizeof(int64_t), s));
  HIP_OK(hipMemsetAsync(out.S.rowptr, 0, sizeof(int64_t), s));
  if (n) k_p_counts<<<nblocks(n, 256), 256, 0, s>>>(D.st, D.s_cnt, n, out.N.rowptr, out.S.rowptr);
  scan_inclusive(out.N.rowptr + 1, n, s, ar);
  scan_inclusive(out.S.rowptr + 1, n, s, ar);
  int64_t* q = ar.alloc<int64_t>(5);
  k_coarse_summary<<<1, 64, 0, s>>>(D.meta, out.N.rowptr + n, out.S.rowptr + n, q);
  // (before the read-back: a copy to pageable host memory returns only
  // once the copy, and so everything queued before it, is done)
  if (overlap) overlap();
  int64_t hq[5];
  read_back(hq, q, sizeof(hq), s);
  if (hq[2] & DERR_PATTERN) throw Error(EMIN_ERR_PATTERN, "given C points unsorted or out of range");
  if (hq[2] & DERR_CAPACITY) throw Error(EMIN_ERR_CAPACITY, "alg3: S set or BFS ball capacity");
  out.n_c = hq[0];
  out.n_alg3 = hq[1];
  out.N.nnz = hq[3];
  out.S.nnz = hq[4];
  out.N.ncols = out.n_c;
  out.cid = ar.alloc<int32_t>(n);
  out.clist = ar.alloc<int32_t>(out.n_c);
  if (n) k_compact<<<nblocks(n, 256), 256, 0, s>>>(incl, D.st, n, out.clist, out.cid);
  out.N.col = ar.alloc<int32_t>(out.N.nnz);
  out.S.col = ar.alloc<int32_t>(out.S.nnz);
  out.sdist = ar.alloc<uint8_t>(out.S.nnz);
  if (n)
    k_p_fill<<<nblocks(n, 256), 256, 0, s>>>(D, out.cid, out.N.rowptr, out.N.col, out.S.rowptr,
                                              out.S.col, out.sdist);
}

}  // namespace emin
