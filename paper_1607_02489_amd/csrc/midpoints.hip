// Alg. 4 (find_velocity_Cpoints): pressure mid-points.
//
// Every F vertex i with |S_i| >= 2 gets, in parallel, its target X_i (the
// barycentre of S_i), its search set B_i = {j in F : S_i subset of S_j}, the
// closest vertex m_i, and the set T_i of vertices of B_i that are closer to
// m_i than tau2 * t_i (t_i the diagonal of B_i's bounding box).  T_i has no
// fixed size: a count pass, a scan and a fill pass store the sets as one CSR.
// The loop of Alg. 4 then reduces to: visiting i in the order (|S_i| desc,
// i asc), add m_i to C-bar unless some vertex of T_i is already in C-bar.
// That ordered pass runs in one wave with C-bar as a bitmap in LDS, 64
// entries at a time: each entry's dependence on the earlier entries of its
// chunk is a 64-bit mask, resolved in lane order.
#include "coarsen.h"
#include "prof.h"

namespace emin {

// entries of T_i the ordered pass keeps in registers; longer sets are read
// from the CSR for the rest
constexpr int TPRE = 8;

__device__ __forceinline__ bool subset_sorted(const int32_t* a, int na, const int32_t* b, int nb) {
  int q = 0;
  for (int p = 0; p < na; p++) {
    while (q < nb && b[q] < a[p]) q++;
    if (q >= nb || b[q] != a[p]) return false;
    q++;
  }
  return true;
}

// Candidate e of B_i's search list (the vertices whose S holds S_i's first
// C point) is in T_i: an F vertex whose S contains S_i, within the
// closeness radius of m (squared distance below thr).
__device__ __forceinline__ bool in_closeness_set(int64_t e, int64_t t1, int32_t m, double thr,
                                                 const int32_t* tcol, const int64_t* srp,
                                                 const int32_t* scol, int64_t s0, int si,
                                                 const uint8_t* st, const double* x, int dim) {
  if (e >= t1 || m < 0) return false;
  const int32_t j = tcol[e];
  if (st[j] == ST_C ||
      !subset_sorted(scol + s0, si, scol + srp[j], (int)(srp[j + 1] - srp[j])))
    return false;
  double d2 = 0.0;
  for (int d = 0; d < dim; d++) {
    const double r = x[(int64_t)j * dim + d] - x[(int64_t)m * dim + d];
    d2 = d2 + r * r;
  }
  return d2 < thr;
}

// One wave per F vertex i: X_i (mean of S_i's coordinates, summed in S
// order), B_i = {j in F : S_i within S_j} (candidates j: the F vertices whose
// S contains S_i's first C point), m = argmin over B_i of (|x_j - X_i|^2, j),
// w2 = squared diagonal of B_i's bounding box, and the size of T_i = {j in
// B_i : |x_j - x_m|^2 < tau2^2 w2} (written to tcnt[i], the count array of
// T's CSR; the closeness threshold goes to thr_out).  The lanes share the
// candidates; minima and box by wave reductions (exact).
__global__ __launch_bounds__(256) void k_mid_prep(const int64_t* srp, const int32_t* scol,
                                                  const int64_t* trp, const int32_t* tcol,
                                                  const uint8_t* st, const double* x, int dim,
                                                  double tau2_sq, int64_t n, int32_t* m_out,
                                                  int32_t* size_key, int64_t* tcnt,
                                                  double* thr_out) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;   // whole wave
  const int64_t s0 = srp[i], s1 = srp[i + 1];
  const int si = (int)(s1 - s0);
  if (st[i] == ST_C || si < 2) {
    if (lane == 0) { m_out[i] = -1; size_key[i] = 0; tcnt[i] = 0; }
    return;
  }
  double X[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < dim; d++) {
    double acc = 0.0;
    for (int64_t e = s0; e < s1; e++) acc = acc + x[(int64_t)scol[e] * dim + d];
    X[d] = acc / (double)si;
  }
  const int32_t c0 = scol[s0];
  const int64_t t0 = trp[c0], t1 = trp[c0 + 1];
  const double INF = __builtin_inf();
  double mk = INF;
  int32_t mi = INT32_MAX;
  double lo[3] = {INF, INF, INF}, hi[3] = {-INF, -INF, -INF};
  for (int64_t e = t0 + lane; e < t1; e += 64) {
    const int32_t j = tcol[e];
    if (st[j] == ST_C) continue;
    if (!subset_sorted(scol + s0, si, scol + srp[j], (int)(srp[j + 1] - srp[j]))) continue;
    double d2 = 0.0;
    for (int d = 0; d < dim; d++) {
      const double r = x[(int64_t)j * dim + d] - X[d];
      d2 = d2 + r * r;
    }
    if (d2 < mk || (d2 == mk && j < mi)) { mk = d2; mi = j; }
    for (int d = 0; d < dim; d++) {
      const double v = x[(int64_t)j * dim + d];
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
    }
  }
  wave_argmin(mk, mi);
  for (int d = 0; d < dim; d++) {
    lo[d] = wave_min_f64(lo[d]);
    hi[d] = -wave_min_f64(-hi[d]);
  }
  const int32_t m = mi == INT32_MAX ? -1 : mi;   // i itself is in B_i, so m exists
  double w2 = 0.0;
  for (int d = 0; d < dim; d++) {
    const double w = hi[d] - lo[d];
    w2 = w2 + w * w;
  }
  const double thr = tau2_sq * w2;
  int64_t tc = 0;   // wave-uniform running count
  for (int64_t e0 = t0; e0 < t1; e0 += 64)
    tc += __popcll(__ballot(in_closeness_set(e0 + lane, t1, m, thr, tcol, srp, scol, s0, si,
                                             st, x, dim)));
  if (lane == 0) {
    m_out[i] = m;
    size_key[i] = si;
    tcnt[i] = tc;
    thr_out[i] = thr;
  }
}

// T_i in candidate order into its CSR row (the same test as the count pass).
__global__ __launch_bounds__(256) void k_mid_tfill(const int64_t* srp, const int32_t* scol,
                                                   const int64_t* trp, const int32_t* tcol,
                                                   const uint8_t* st, const double* x, int dim,
                                                   int64_t n, const int32_t* m_in,
                                                   const double* thr_in, const int64_t* toff,
                                                   int32_t* tlist) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;   // whole wave
  const int64_t base = toff[i], len = toff[i + 1] - base;
  if (len == 0) return;
  const int64_t s0 = srp[i];
  const int si = (int)(srp[i + 1] - s0);
  const int32_t m = m_in[i];
  const double thr = thr_in[i];
  const int32_t c0 = scol[s0];
  const int64_t t0 = trp[c0], t1 = trp[c0 + 1];
  int64_t tc = 0;
  for (int64_t e0 = t0; e0 < t1; e0 += 64) {
    const int64_t e = e0 + lane;
    const bool in_t = in_closeness_set(e, t1, m, thr, tcol, srp, scol, s0, si, st, x, dim);
    const unsigned long long bal = __ballot(in_t);
    const int64_t p = tc + __popcll(bal & ((1ull << lane) - 1ull));
    if (in_t && p < len) tlist[base + p] = tcol[e];
    tc += __popcll(bal);
  }
}

// Visiting order of Alg. 4 as one stable counting sort: class c = KMAX - |S|
// (|S| from KMAX down to 2), ascending index within a class.  Per block (256
// vertices) and class the count (class-major), one inclusive scan gives each
// block's start, and per-wave ballots rank the vertices inside the block.
constexpr int KMAX = 32;             // S sets hold at most 32 entries
constexpr int NCLS = KMAX - 1;       // |S| = 32 ... 2

__global__ __launch_bounds__(256) void k_order_count(const int32_t* key, int64_t n, int64_t nb,
                                                    int64_t* bc, int* err) {
  __shared__ int cnt[NCLS];
  if (threadIdx.x < NCLS) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = i < n ? key[i] : 0;
  if (k >= 2 && k <= KMAX) atomicAdd(&cnt[KMAX - k], 1);
  else if (k > KMAX) atomicOr(err, DERR_CAPACITY);
  __syncthreads();
  if (threadIdx.x < NCLS) bc[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_order_place(const int32_t* key, int64_t n,
                                                    const int64_t* incl, int64_t nb,
                                                    int32_t* order) {
  __shared__ int wc[4][NCLS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = i < n ? key[i] : 0;
  const int c = (k >= 2 && k <= KMAX) ? KMAX - k : -1;
  uint64_t mine = 0;
  for (int q = 0; q < NCLS; q++) {
    const uint64_t m = __ballot(c == q);
    if (lane == 0) wc[w][q] = __popcll(m);
    if (c == q) mine = m;
  }
  __syncthreads();
  if (c < 0) return;
  const int64_t kk = (int64_t)c * nb + blockIdx.x;
  int64_t pos = kk ? incl[kk - 1] : 0;
  for (int v = 0; v < w; v++) pos += wc[v][c];
  order[pos + __popcll(mine & ((1ull << lane) - 1ull))] = (int32_t)i;
}

__global__ void k_order_total(const int64_t* incl, int64_t len, const int* err,
                              const int64_t* ttot, int64_t* out) {
  if (threadIdx.x == 0) {
    out[0] = len ? incl[len - 1] : 0;
    out[1] = *err;
    out[2] = *ttot;
  }
}

// per position p of the visiting order: m, the first TPRE entries of T
// (padded with -1), and where the whole of T lies in the CSR (its start and
// length), for sets longer than TPRE
__global__ void k_mid_pack(const int32_t* order, int64_t norder, const int32_t* m,
                           const int64_t* toff, const int32_t* tlist, int32_t* mo, int32_t* to,
                           int64_t* tb, int32_t* tn) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= norder) return;
  const int32_t i = order[p];
  mo[p] = m[i];
  const int64_t a = toff[i];
  const int64_t len = toff[i + 1] - a;
  for (int t = 0; t < TPRE; t++) to[p * TPRE + t] = t < len ? tlist[a + t] : -1;
  tb[p] = a;
  tn[p] = (int32_t)len;
}

// mask of the earlier entries of p's 64-chunk whose m lies in T_p
__global__ void k_mid_dep(const int32_t* mo, const int64_t* tb, const int32_t* tn,
                          const int32_t* tlist, int64_t norder, unsigned long long* dep) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= norder) return;
  const int64_t base = p & ~int64_t(63);
  const int64_t a = tb[p];
  const int len = tn[p];
  unsigned long long d = 0ull;
  for (int t = 0; t < len; t++) {
    const int32_t v = tlist[a + t];
    for (int64_t q = base; q < p; q++)
      if (mo[q] == v) d |= 1ull << (q - base);
  }
  dep[p] = d;
}

// C-bar as a bitmap of 32-bit words: built from the C points in parallel,
// carried through the ordered pass in LDS, expanded to flags afterwards.
__global__ void k_cbits_init(const uint8_t* st, int64_t n, uint32_t* gb) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w * 32 >= n) return;
  uint32_t m = 0u;
  for (int b = 0; b < 32; b++) {
    const int64_t i = w * 32 + b;
    if (i < n && st[i] == ST_C) m |= 1u << b;
  }
  gb[w] = m;
}

__global__ void k_cbits_expand(const uint32_t* gb, int64_t n, uint8_t* cbar,
                               unsigned long long* count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t f = (uint8_t)((gb[i >> 5] >> (i & 31)) & 1u);
  cbar[i] = f;
  const unsigned long long c = __ballot(f != 0);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)__popcll(c));
}

// The ordered pass of Alg. 4 in one wave, 64 entries per chunk.  An entry is
// rejected when some vertex of its T is in C-bar from an earlier chunk (LDS
// bitmap) or is the m of an earlier accepted entry of its own chunk (its
// dependence mask).  Entries without a dependence are decided at once; those
// with one are resolved in rounds along their dependence chains.
__global__ __launch_bounds__(64) void k_mid_decide(const int32_t* mo, const int32_t* to,
                                                   const int64_t* tb, const int32_t* tn,
                                                   const int32_t* tlist,
                                                   const unsigned long long* dep, int64_t norder,
                                                   int64_t n, uint32_t* gb) {
  extern __shared__ uint32_t bits[];
  const int lane = threadIdx.x;
  const int64_t nw = (n + 31) / 32;
  for (int64_t w0 = 0; w0 < nw; w0 += 8 * 64) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int64_t w = w0 + j * 64 + lane;
      v[j] = w < nw ? gb[w] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int64_t w = w0 + j * 64 + lane;
      if (w < nw) bits[w] = v[j];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // software pipeline: each chunk's entries are loaded DEPTH chunks ahead
  // (a chunk's work is far shorter than a memory round trip)
  struct Chunk {
    int32_t T[TPRE];
    int32_t m;
    int32_t len;
    unsigned long long d;
  };
  auto load = [&](int64_t base, Chunk& c) {
    const int64_t p = base + lane;
    const bool ok = p < norder;
#pragma unroll
    for (int t = 0; t < TPRE; t++) c.T[t] = ok ? to[p * TPRE + t] : -1;
    c.m = ok ? mo[p] : -1;
    c.len = ok ? tn[p] : 0;
    c.d = ok ? dep[p] : 0ull;
  };
  auto decide = [&](int64_t base, const Chunk& c) {
    const bool valid = base + lane < norder;
    // the first TPRE bitmap words read together
    uint32_t wd[TPRE];
#pragma unroll
    for (int t = 0; t < TPRE; t++) wd[t] = bits[(c.T[t] >= 0 ? c.T[t] : 0) >> 5];
    bool pre = !valid;
#pragma unroll
    for (int t = 0; t < TPRE; t++)
      if (c.T[t] >= 0 && ((wd[t] >> (c.T[t] & 31)) & 1u)) pre = true;
    // the rest of a longer T from the CSR (large tau2 only)
    if (valid && c.len > TPRE) {
      const int64_t a = tb[base + lane];
      for (int t = TPRE; t < c.len && !pre; t++) {
        const int32_t v = tlist[a + t];
        if ((bits[v >> 5] >> (v & 31)) & 1u) pre = true;
      }
    }
    const unsigned long long rejected = __ballot(pre);
    const unsigned long long depend = __ballot(!pre && c.d != 0ull);
    unsigned long long accepted = ~rejected & ~depend;
    // entries with a dependence (only on earlier lanes) decide in rounds: an
    // entry whose dependences are all decided is accepted iff none of them
    // was; the lowest undecided entry can always decide, and each decision
    // is the one the lane-order pass would make
    unsigned long long decided = ~depend;
    while (decided != ~0ull) {
      const bool mine = !((decided >> lane) & 1ull);
      const bool can = mine && (c.d & ~decided) == 0ull;
      const bool acc = can && (c.d & accepted) == 0ull;
      accepted |= __ballot(acc);
      decided |= __ballot(can);
    }
    if ((accepted >> lane) & 1ull) atomicOr(&bits[c.m >> 5], 1u << (c.m & 31));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  constexpr int DEPTH = 8;
  Chunk c[DEPTH];
#pragma unroll
  for (int k = 0; k < DEPTH; k++) load(64 * k, c[k]);
  for (int64_t base = 0; base < norder; base += 64 * DEPTH) {
#pragma unroll
    for (int k = 0; k < DEPTH; k++) {   // unrolled: every c[k] stays in registers
      if (base + 64 * k < norder) {
        decide(base + 64 * k, c[k]);
        load(base + 64 * (k + DEPTH), c[k]);
      }
    }
  }
  for (int64_t w = lane; w < nw; w += 64) gb[w] = bits[w];
}

int64_t midpoints(const Csr& S, const uint8_t* st, const double* x, int dim, double tau2_sq,
                  uint8_t* cbar, hipStream_t s, Arena& ar, int lds_max) {
  const int64_t n = S.nrows;
  if (n == 0) return 0;
  Csr ST;
  int32_t* tsrc = nullptr;
  transpose_pattern(view(S), ST, tsrc, s, ar);
  int32_t* m = ar.alloc<int32_t>(n);
  int32_t* key = ar.alloc<int32_t>(n);
  double* thr = ar.alloc<double>(n);
  int64_t* toff = ar.alloc<int64_t>(n + 1);   // CSR of the T sets
  int* err = ar.alloc<int>(1);
  HIP_OK(hipMemsetAsync(err, 0, sizeof(int), s));
  HIP_OK(hipMemsetAsync(toff, 0, sizeof(int64_t), s));
  k_mid_prep<<<nblocks(n, 4), 256, 0, s>>>(S.rowptr, S.col, ST.rowptr, ST.col, st, x, dim,
                                            tau2_sq, n, m, key, toff + 1, thr);
  scan_inclusive(toff + 1, n, s, ar);
  // visiting order: |S| descending, index ascending (one read-back with the
  // capacity flag and the total size of the T sets)
  int32_t* order = ar.alloc<int32_t>(n);
  const int64_t nb = (int64_t)nblocks(n, 256);
  int64_t* bc = ar.alloc<int64_t>((size_t)NCLS * nb);
  int64_t* tot = ar.alloc<int64_t>(3);
  k_order_count<<<(unsigned)nb, 256, 0, s>>>(key, n, nb, bc, err);
  scan_inclusive(bc, NCLS * nb, s, ar);
  k_order_place<<<(unsigned)nb, 256, 0, s>>>(key, n, bc, nb, order);
  k_order_total<<<1, 64, 0, s>>>(bc, NCLS * nb, err, toff + n, tot);
  int64_t th[3];
  read_back(th, tot, sizeof(th), s);
  if (th[1]) throw Error(EMIN_ERR_CAPACITY, "alg4: S set longer than 32");
  const int64_t norder = th[0];
  const int64_t ttot = th[2];
  const size_t lds = (size_t)((n + 31) / 32) * 4;
  if ((int64_t)lds > lds_max) throw Error(EMIN_ERR_CAPACITY, "alg4: C-bar bitmap exceeds LDS");
  allow_lds((const void*)k_mid_decide);
  int32_t* tlist = ar.alloc<int32_t>((size_t)(ttot > 0 ? ttot : 1));
  if (ttot)
    k_mid_tfill<<<nblocks(n, 4), 256, 0, s>>>(S.rowptr, S.col, ST.rowptr, ST.col, st, x, dim, n,
                                               m, thr, toff, tlist);
  int32_t* mo = ar.alloc<int32_t>(norder);
  int32_t* to = ar.alloc<int32_t>((size_t)norder * TPRE);
  int64_t* tb = ar.alloc<int64_t>(norder);
  int32_t* tn = ar.alloc<int32_t>(norder);
  unsigned long long* dep = ar.alloc<unsigned long long>(norder);
  if (norder) {
    k_mid_pack<<<nblocks(norder, 256), 256, 0, s>>>(order, norder, m, toff, tlist, mo, to, tb,
                                                     tn);
    k_mid_dep<<<nblocks(norder, 256), 256, 0, s>>>(mo, tb, tn, tlist, norder, dep);
  }
  const int64_t nw = (n + 31) / 32;
  uint32_t* gb = ar.alloc<uint32_t>(nw);
  k_cbits_init<<<nblocks(nw, 256), 256, 0, s>>>(st, n, gb);
  {
    prof::Scope ps(s, EMIN_PROF_ALG4, 0.0);
    k_mid_decide<<<1, 64, lds, s>>>(mo, to, tb, tn, tlist, dep, norder, n, gb);
  }
  HIP_OK(hipGetLastError());
  unsigned long long* c = ar.alloc<unsigned long long>(2);
  HIP_OK(hipMemsetAsync(c, 0, 2 * sizeof(unsigned long long), s));
  k_cbits_expand<<<nblocks(n, 256), 256, 0, s>>>(gb, n, cbar, c);
  return (int64_t)d2h(c, s);
}

}  // namespace emin
