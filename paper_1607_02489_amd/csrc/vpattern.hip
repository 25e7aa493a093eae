// sec. 4.2: coarse velocities and the velocity sparsity pattern.
//
// Row i of N^(v) holds every C^(v) node within graph distance 3 of i in the
// nodal graph of the filtered velocity block.  The search runs from the C
// points (far fewer than the nodes): one wave per source walks its
// distance-3 ball with an LDS hash set and appends the source to each row it
// reaches.  Rows are sorted afterwards, so the atomic append order does not
// show.  Extra C^(v) points (non-Dirichlet F nodes with no C^(v) within
// distance 3, taken in ascending order) are found in parallel as the ordered
// independent set described at k_vconf.
#include "coarsen.h"
#include "prof.h"

namespace emin {

constexpr int VCAP = 64;      // max C^(v) per pattern row
constexpr int VB_WAVES = 2;   // waves (sources) per block
constexpr int VHASH = 2048;   // LDS hash slots per wave
constexpr int VBALL = 2048;   // ball list per wave

__device__ __forceinline__ uint32_t vhash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// The distance-3 ball of c in the wave's LDS list ball[0..nb): breadth-first
// over the graph with an LDS hash set of the visited vertices.  Returns the
// list length; *bad is set when the hash set or the list overflows.
__device__ int wave_ball3(const int64_t* grp, const int32_t* gcol, int32_t c, int32_t* hs,
                          int32_t* ball, int* nb, int lane, bool* bad) {
  for (int t = lane; t < VHASH; t += 64) hs[t] = -1;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane == 0) {
    ball[0] = c;
    hs[vhash((uint32_t)c) & (VHASH - 1)] = c;
    *nb = 1;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int ls = 0, le = 1;
  for (int L = 0; L < 3; L++) {
    for (int f = ls + lane; f < le; f += 64) {
      const int32_t v = ball[f];
      for (int64_t e = grp[v]; e < grp[v + 1]; e++) {
        const int32_t u = gcol[e];
        if (u == v) continue;
        uint32_t h = vhash((uint32_t)u) & (VHASH - 1);
        int probes = 0;
        while (true) {
          const int32_t old = atomicCAS(&hs[h], -1, u);
          if (old == -1) {
            const int p = atomicAdd(nb, 1);
            if (p < VBALL) ball[p] = u; else *bad = true;
            break;
          }
          if (old == u) break;
          h = (h + 1) & (VHASH - 1);
          if (++probes >= VHASH / 2) { *bad = true; break; }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    ls = le;
    le = min(*nb, VBALL);
  }
  return le;
}

// one wave per source c: mark its distance-3 ball covered and append c to
// the rows it reaches (sources srcs[0..nsrc), or [0..*dcount) when dcount
// is given)
__global__ __launch_bounds__(64 * VB_WAVES) void k_vbfs(const int64_t* grp, const int32_t* gcol,
                                                        const int32_t* srcs, int64_t nsrc,
                                                        const int64_t* dcount,
                                                        const uint8_t* dir, uint8_t* cov,
                                                        int32_t* vcnt, int32_t* vbuf, int* err) {
  __shared__ int32_t hash_all[VB_WAVES][VHASH];
  __shared__ int32_t ball_all[VB_WAVES][VBALL];
  __shared__ int nb_all[VB_WAVES];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t si = (int64_t)blockIdx.x * VB_WAVES + w;
  if (si >= nsrc || (dcount && si >= *dcount)) return;
  int32_t* ball = ball_all[w];
  const int32_t c = srcs[si];
  bool bad = false;
  const int le = wave_ball3(grp, gcol, c, hash_all[w], ball, &nb_all[w], lane, &bad);
  if (bad) atomicOr(err, DERR_CAPACITY);
  for (int t = lane; t < le; t += 64) {
    const int32_t v = ball[t];
    cov[v] = 1;
    if (v != c && !dir[v]) {
      const int slot = atomicAdd(&vcnt[v], 1);
      if (slot < VCAP) vbuf[(int64_t)v * VCAP + slot] = c;
      else atomicOr(err, DERR_CAPACITY);
    }
  }
}

// Extra C^(v) (sec. 4.2): taken in ascending order, each one covering its
// distance-3 ball, among the eligible vertices (not C, not Dirichlet, not
// covered by the C^(v) balls).  Vertex j is taken exactly when no smaller
// taken vertex has j in its ball: the set is the lexicographically first
// maximal independent set of the eligible vertices under "e reaches j within
// distance 3".  It is computed in parallel with the same result: each
// eligible e lists the smaller eligible vertices whose balls hold it
// (k_vconf, one wave per eligible source, which appends itself to the lists
// of the larger eligible vertices in its ball), then k_lfmis decides the
// vertices in rounds: one is taken once every vertex on its list is decided
// out, and is out once one on its list is taken.  The smallest undecided
// vertex is decided in every round, so the rounds end.

// the ball of eligible source ei: append ei to the list of every larger
// eligible vertex in it (count pass: cnt; fill pass: col at rp + cursor)
template <bool FILL>
__global__ __launch_bounds__(64 * VB_WAVES) void k_vconf(const int64_t* grp, const int32_t* gcol,
                                                         const int32_t* elist, int64_t m,
                                                         const int32_t* eid, int32_t* cnt,
                                                         const int64_t* rp, int32_t* col,
                                                         int* err) {
  __shared__ int32_t hash_all[VB_WAVES][VHASH];
  __shared__ int32_t ball_all[VB_WAVES][VBALL];
  __shared__ int nb_all[VB_WAVES];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ei = (int64_t)blockIdx.x * VB_WAVES + w;
  if (ei >= m) return;
  int32_t* ball = ball_all[w];
  const int32_t c = elist[ei];
  bool bad = false;
  const int le = wave_ball3(grp, gcol, c, hash_all[w], ball, &nb_all[w], lane, &bad);
  if (bad) atomicOr(err, DERR_CAPACITY);
  for (int t = lane; t < le; t += 64) {
    const int32_t v = ball[t];
    const int32_t k = eid[v];
    if (v <= c || k < 0) continue;
    const int slot = atomicAdd(&cnt[k], 1);
    // (a ball cut short by an overflow may differ between the passes; the
    // overflow is reported, and the fill stays inside the counted room)
    if (FILL && rp[k] + slot < rp[k + 1]) col[rp[k] + slot] = (int32_t)ei;
  }
}

// Rounds of the ordered independent set over the conflict lists, one
// workgroup; state 0 undecided, 1 taken, 2 out.  States live in LDS when
// they fit (lds), else in global memory read and written with agent-scope
// atomics.
template <bool LDS>
__global__ __launch_bounds__(1024) void k_lfmis(const int64_t* rp, const int32_t* col, int64_t m,
                                                uint8_t* gstate, const int32_t* elist,
                                                uint8_t* cv, int32_t* out_taken) {
  extern __shared__ uint8_t sstate[];
  __shared__ int pending_sh, taken_sh;
  uint8_t* st = LDS ? sstate : gstate;
  const int tid = threadIdx.x;
  auto ld = [&](int64_t i) -> uint8_t {
    if (LDS) return __hip_atomic_load(&st[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return __hip_atomic_load(&st[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto stv = [&](int64_t i, uint8_t v) {
    if (LDS) __hip_atomic_store(&st[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else __hip_atomic_store(&st[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  for (int64_t i = tid; i < m; i += 1024) stv(i, 0);
  if (tid == 0) taken_sh = 0;
  __syncthreads();
  while (true) {
    if (tid == 0) pending_sh = 0;
    __syncthreads();
    bool pend = false;
    for (int64_t i = tid; i < m; i += 1024) {
      if (ld(i) != 0) continue;
      bool all_out = true, any_in = false;
      for (int64_t t = rp[i]; t < rp[i + 1]; t++) {
        const uint8_t s = ld(col[t]);
        if (s == 1) { any_in = true; break; }
        if (s == 0) all_out = false;
      }
      if (any_in) stv(i, 2);
      else if (all_out) stv(i, 1);
      else pend = true;
    }
    if (pend) pending_sh = 1;
    __syncthreads();
    const int more = pending_sh;
    __syncthreads();
    if (!more) break;
  }
  int tk = 0;
  for (int64_t i = tid; i < m; i += 1024)
    if (ld(i) == 1) {
      cv[elist[i]] = 1;
      tk++;
    }
  atomicAdd(&taken_sh, tk);
  __syncthreads();
  if (tid == 0) *out_taken = taken_sh;
}

__global__ void k_elig_flags(const uint8_t* cv, const uint8_t* dir, const uint8_t* cov,
                             int64_t n, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = !cv[i] && !dir[i] && !cov[i];
}

__global__ void k_elig_compact(const int64_t* incl, const uint8_t* cv, const uint8_t* dir,
                               const uint8_t* cov, int64_t n, int32_t* list, int32_t* eid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool e = !cv[i] && !dir[i] && !cov[i];
  const int32_t id = e ? (int32_t)(incl[i] - 1) : -1;
  eid[i] = id;
  if (e) list[id] = (int32_t)i;
}

// the taken vertices (cv set by k_lfmis) in ascending order
__global__ void k_taken_list(const int64_t* incl, const int32_t* elist, const uint8_t* cv,
                             int64_t m, int32_t* extra) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m && cv[elist[i]]) extra[incl[i] - 1] = elist[i];
}

__global__ void k_widen_i32(const int32_t* a, int64_t n, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i];
}

__global__ void k_taken_flags(const int32_t* elist, const uint8_t* cv, int64_t m, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = cv[elist[i]] != 0;
}

// scalars gathered for one read-back into out[0..4] (a null source reads 0)
__global__ void k_gather_scalars(const int64_t* a, const int64_t* b, const unsigned long long* c,
                                 const unsigned long long* d, const int* e, int64_t* out) {
  if (threadIdx.x == 0) {
    out[0] = a ? *a : 0;
    out[1] = b ? *b : 0;
    out[2] = c ? (int64_t)*c : 0;
    out[3] = d ? (int64_t)*d : 0;
    out[4] = e ? *e : 0;
  }
}

__global__ void k_flags_u8(const uint8_t* f, int64_t n, int64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f[i] != 0;
}

__global__ void k_compact_u8(const int64_t* incl, const uint8_t* f, int64_t n, int32_t* list,
                             int32_t* cid) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t id = f[i] ? (int32_t)(incl[i] - 1) : -1;
  if (cid) cid[i] = id;
  if (f[i]) list[id] = (int32_t)i;
}

__global__ void k_v_counts(const uint8_t* cv, const uint8_t* dir, const int32_t* vcnt, int64_t n,
                           int64_t* rp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rp[i + 1] = cv[i] ? 1 : (dir[i] ? 0 : vcnt[i]);
}

// row i of N^(v): {itself} for a C^(v) node, nothing for a Dirichlet node,
// else the coarse numbers of the C^(v) that reached it, ascending (distinct
// sources, so the rank of a source among the row's gives its place); G
// lanes per row
template <int G>
__global__ __launch_bounds__(256) void k_v_fill(const uint8_t* cv, const uint8_t* dir,
                                               const int32_t* vcnt, const int32_t* vbuf,
                                               const int32_t* cid, int64_t n, const int64_t* rp,
                                               int32_t* col) {
  const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (i >= n) return;
  const int64_t p = rp[i];
  if (cv[i]) {
    if (lane == 0) col[p] = cid[i];
    return;
  }
  if (dir[i]) return;
  const int32_t* b = vbuf + i * VCAP;
  const int m = vcnt[i];
  for (int t = lane; t < m; t += G) {
    const int32_t key = b[t];
    int rank = 0;
    for (int u = 0; u < m; u++) rank += b[u] < key;
    col[p + rank] = cid[key];
  }
}

void velocity_pattern(const Csr& G, const uint8_t* dir, uint8_t* cv, VPatternOut& out,
                      hipStream_t s, Arena& ar, int lds_max) {
  const int64_t n = G.nrows;
  int* err = ar.alloc<int>(1);
  HIP_OK(hipMemsetAsync(err, 0, sizeof(int), s));
  uint8_t* cov = ar.alloc<uint8_t>(n);
  int32_t* vcnt = ar.alloc<int32_t>(n);
  int32_t* vbuf = ar.alloc<int32_t>((size_t)n * VCAP);
  HIP_OK(hipMemsetAsync(cov, 0, n, s));
  HIP_OK(hipMemsetAsync(vcnt, 0, sizeof(int32_t) * n, s));
  // initial C^(v) list
  int64_t* incl = ar.alloc<int64_t>(n + 1);
  int64_t* q = ar.alloc<int64_t>(5);
  if (n) k_flags_u8<<<nblocks(n, 256), 256, 0, s>>>(cv, n, incl);
  scan_inclusive(incl, n, s, ar);
  const int64_t n0 = n ? d2h(incl + n - 1, s) : 0;
  int32_t* src0 = ar.alloc<int32_t>(n0);
  if (n) k_compact_u8<<<nblocks(n, 256), 256, 0, s>>>(incl, cv, n, src0, nullptr);
  if (n0) k_vbfs<<<nblocks(n0, VB_WAVES), 64 * VB_WAVES, 0, s>>>(G.rowptr, G.col, src0, n0, nullptr, dir,
                                                                  cov, vcnt, vbuf, err);
  // extra points: the eligible vertices, their conflict lists, the rounds
  if (n) k_elig_flags<<<nblocks(n, 256), 256, 0, s>>>(cv, dir, cov, n, incl);
  scan_inclusive(incl, n, s, ar);
  const int64_t m = n ? d2h(incl + n - 1, s) : 0;
  if (m) {
    prof::Scope ps(s, EMIN_PROF_VPAT, 0.0);
    int32_t* elist = ar.alloc<int32_t>(m);
    int32_t* eid = ar.alloc<int32_t>(n);
    k_elig_compact<<<nblocks(n, 256), 256, 0, s>>>(incl, cv, dir, cov, n, elist, eid);
    int64_t* crp = ar.alloc<int64_t>(m + 1);
    int32_t* ccnt = ar.alloc<int32_t>(m);
    HIP_OK(hipMemsetAsync(ccnt, 0, sizeof(int32_t) * m, s));
    k_vconf<false><<<nblocks(m, VB_WAVES), 64 * VB_WAVES, 0, s>>>(
        G.rowptr, G.col, elist, m, eid, ccnt, nullptr, nullptr, err);
    HIP_OK(hipMemsetAsync(crp, 0, sizeof(int64_t), s));
    k_widen_i32<<<nblocks(m, 256), 256, 0, s>>>(ccnt, m, crp + 1);
    scan_inclusive(crp + 1, m, s, ar);
    const int64_t nconf = d2h(crp + m, s);
    int32_t* ccol = ar.alloc<int32_t>(nconf > 0 ? nconf : 1);
    HIP_OK(hipMemsetAsync(ccnt, 0, sizeof(int32_t) * m, s));
    k_vconf<true><<<nblocks(m, VB_WAVES), 64 * VB_WAVES, 0, s>>>(
        G.rowptr, G.col, elist, m, eid, ccnt, crp, ccol, err);
    int32_t* ntaken = ar.alloc<int32_t>(1);
    if (m + 64 <= lds_max) {
      allow_lds((const void*)k_lfmis<true>);
      k_lfmis<true><<<1, 1024, (size_t)m, s>>>(crp, ccol, m, nullptr, elist, cv, ntaken);
    } else {
      uint8_t* gst = ar.alloc<uint8_t>(m);
      k_lfmis<false><<<1, 1024, 0, s>>>(crp, ccol, m, gst, elist, cv, ntaken);
    }
    HIP_OK(hipGetLastError());
    // the taken vertices in ascending order; each covers its ball and joins
    // the rows it reaches
    int64_t* tincl = ar.alloc<int64_t>(m);
    k_taken_flags<<<nblocks(m, 256), 256, 0, s>>>(elist, cv, m, tincl);
    scan_inclusive(tincl, m, s, ar);
    int32_t* extra = ar.alloc<int32_t>(m);
    k_taken_list<<<nblocks(m, 256), 256, 0, s>>>(tincl, elist, cv, m, extra);
    k_vbfs<<<nblocks(m, VB_WAVES), 64 * VB_WAVES, 0, s>>>(G.rowptr, G.col, extra, m, tincl + m - 1,
                                                           dir, cov, vcnt, vbuf, err);
  }
  // final numbering and the pattern: C^(v) size, the error flag and the
  // pattern size in one read-back
  if (n) k_flags_u8<<<nblocks(n, 256), 256, 0, s>>>(cv, n, incl);
  scan_inclusive(incl, n, s, ar);
  out.N.nrows = n;
  out.N.rowptr = ar.alloc<int64_t>(n + 1);
  HIP_OK(hipMemsetAsync(out.N.rowptr, 0, sizeof(int64_t), s));
  if (n) k_v_counts<<<nblocks(n, 256), 256, 0, s>>>(cv, dir, vcnt, n, out.N.rowptr);
  scan_inclusive(out.N.rowptr + 1, n, s, ar);
  k_gather_scalars<<<1, 64, 0, s>>>(n ? incl + n - 1 : nullptr, out.N.rowptr + n, nullptr,
                                    nullptr, err, q);
  int64_t hc[5];
  read_back(hc, q, sizeof(hc), s);
  if (hc[4]) throw Error(EMIN_ERR_CAPACITY, "velocity pattern: row or ball capacity");
  out.n_c = hc[0];
  out.n_extra = out.n_c - n0;
  out.N.nnz = hc[1];
  out.N.ncols = out.n_c;
  out.cid = ar.alloc<int32_t>(n);
  out.clist = ar.alloc<int32_t>(out.n_c);
  if (n) k_compact_u8<<<nblocks(n, 256), 256, 0, s>>>(incl, cv, n, out.clist, out.cid);
  out.N.col = ar.alloc<int32_t>(out.N.nnz);
  if (n)
    k_v_fill<8><<<nblocks(n, 32), 256, 0, s>>>(cv, dir, vcnt, vbuf, out.cid, n, out.N.rowptr,
                                                 out.N.col);
}

}  // namespace emin
