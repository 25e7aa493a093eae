// sec. 4.2: coarse velocities and the velocity sparsity pattern.
//
// Row i of N^(v) holds every C^(v) node within graph distance 3 of i in the
// nodal graph of the filtered velocity block.  The search runs from the C
// points (far fewer than the nodes): one wave per source walks its
// distance-3 ball with an LDS hash set and appends the source to each row it
// reaches.  Rows are sorted afterwards, so the atomic append order does not
// show.  Extra C^(v) points (non-Dirichlet F nodes with no C^(v) within
// distance 3) are taken in ascending order by a single workgroup.
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

// one wave per source c: BFS to depth 3, mark covered, append c to the rows
__global__ __launch_bounds__(64 * VB_WAVES) void k_vbfs(const int64_t* grp, const int32_t* gcol,
                                                        const int32_t* srcs, int64_t nsrc,
                                                        const uint8_t* dir, uint8_t* cov,
                                                        int32_t* vcnt, int32_t* vbuf, int* err) {
  __shared__ int32_t hash_all[VB_WAVES][VHASH];
  __shared__ int32_t ball_all[VB_WAVES][VBALL];
  __shared__ int nb_all[VB_WAVES];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t si = (int64_t)blockIdx.x * VB_WAVES + w;
  if (si >= nsrc) return;
  int32_t* hs = hash_all[w];
  int32_t* ball = ball_all[w];
  for (int t = lane; t < VHASH; t += 64) hs[t] = -1;
  const int32_t c = srcs[si];
  if (lane == 0) {
    ball[0] = c;
    hs[vhash((uint32_t)c) & (VHASH - 1)] = c;
    nb_all[w] = 1;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int ls = 0, le = 1;
  bool bad = false;
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
            const int p = atomicAdd(&nb_all[w], 1);
            if (p < VBALL) ball[p] = u; else bad = true;
            break;
          }
          if (old == u) break;
          h = (h + 1) & (VHASH - 1);
          if (++probes >= VHASH / 2) { bad = true; break; }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    ls = le;
    le = min(nb_all[w], VBALL);
  }
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

// Extra C^(v), ascending: the smallest non-Dirichlet, uncovered, non-C node
// at or after the cursor is converted, then its distance-3 ball is covered.
// Visited marks: with nwin > 0, a bitmap in LDS over the index window
// j ± 3·bw of the ball (bw = the graph's index bandwidth), cleared per ball;
// otherwise per-vertex stamps in global memory.
__global__ __launch_bounds__(1024) void k_vextras(const int64_t* grp, const int32_t* gcol,
                                                  int64_t n, const uint8_t* dir, uint8_t* cv,
                                                  uint8_t* cov, int32_t* vis, int32_t* extra,
                                                  int32_t* nextra, int ballcap, int deg_cap,
                                                  int64_t bw, int nwin, int* err) {
  extern __shared__ int32_t ball[];
  uint32_t* win = reinterpret_cast<uint32_t*>(ball + ballcap);
  __shared__ int found_sh, nb_sh, ne_sh, bad_sh;
  const int tid = threadIdx.x;
  if (tid == 0) { ne_sh = 0; bad_sh = 0; }
  int64_t cursor = 0;
  int32_t stamp = 0;
  while (true) {
    if (tid == 0) found_sh = INT32_MAX;
    __syncthreads();
    // eight flags per thread per pass (vertices before the cursor are never
    // eligible again, so the pass may start at the aligned position below it)
    for (int64_t base = cursor & ~(int64_t)7; base < n; base += 8 * 1024) {
      const int64_t v0 = base + (int64_t)tid * 8;
      int f = INT32_MAX;
      if (v0 + 8 <= n) {
        const uint64_t bad = *reinterpret_cast<const uint64_t*>(cv + v0) |
                             *reinterpret_cast<const uint64_t*>(dir + v0) |
                             *reinterpret_cast<const uint64_t*>(cov + v0);
        for (int q = 0; q < 8; q++)
          if (((bad >> (8 * q)) & 0xFFu) == 0u) { f = (int)(v0 + q); break; }
      } else {
        for (int64_t v = v0; v < n; v++)
          if (!cv[v] && !dir[v] && !cov[v]) { f = (int)v; break; }
      }
      if (f != INT32_MAX) atomicMin(&found_sh, f);
      __syncthreads();
      const int ff = found_sh;
      __syncthreads();
      if (ff != INT32_MAX) break;
    }
    const int j = found_sh;
    if (j == INT32_MAX) break;
    const int64_t lo = (int64_t)j - 3 * bw > 0 ? (int64_t)j - 3 * bw : 0;
    if (nwin) {
      for (int t = tid; t < nwin; t += 1024) win[t] = 0u;
      __syncthreads();
    }
    if (tid == 0) {
      cv[j] = 1;
      extra[ne_sh] = j;
      ne_sh++;
      ball[0] = j;
      if (nwin) {
        const int64_t o = j - lo;
        win[o >> 5] |= 1u << (o & 31);
      } else {
        atomicMax(&vis[j], stamp);
      }
      nb_sh = 1;
    }
    __syncthreads();
    int ls = 0, le = 1;
    const int per = 1024 / deg_cap;
    for (int L = 0; L < 3; L++) {
      for (int base = ls; base < le; base += per) {
        const int f = base + tid / deg_cap;
        const int slot = tid % deg_cap;
        if (f < le) {
          const int32_t v = ball[f];
          for (int64_t e = grp[v] + slot; e < grp[v + 1]; e += deg_cap) {
            const int32_t u = gcol[e];
            if (u == v) continue;
            bool fresh;
            if (nwin) {
              const int64_t o = (int64_t)u - lo;
              const uint32_t bit = 1u << (o & 31);
              fresh = (atomicOr(&win[o >> 5], bit) & bit) == 0u;
            } else {
              fresh = atomicMax(&vis[u], stamp) < stamp;
            }
            if (fresh) {
              const int p = atomicAdd(&nb_sh, 1);
              if (p < ballcap) ball[p] = u; else atomicOr(&bad_sh, 1);
            }
          }
        }
      }
      __syncthreads();
      ls = le;
      le = min(nb_sh, ballcap);
      __syncthreads();
    }
    for (int t = tid; t < le; t += 1024) cov[ball[t]] = 1;
    __syncthreads();
    stamp++;
    cursor = (int64_t)j + 1;
    if (bad_sh) break;
  }
  if (tid == 0) {
    *nextra = ne_sh;
    if (bad_sh) atomicOr(err, DERR_CAPACITY);
  }
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

__global__ void k_v_fill(const uint8_t* cv, const uint8_t* dir, int32_t* vcnt, int32_t* vbuf,
                         const int32_t* cid, int64_t n, const int64_t* rp, int32_t* col) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = rp[i];
  if (cv[i]) { col[p] = cid[i]; return; }
  if (dir[i]) return;
  int32_t* b = vbuf + i * VCAP;
  const int m = vcnt[i];
  for (int a = 1; a < m; a++) {
    const int32_t key = b[a];
    int q = a;
    while (q > 0 && b[q - 1] > key) { b[q] = b[q - 1]; q--; }
    b[q] = key;
  }
  for (int a = 0; a < m; a++) col[p + a] = cid[b[a]];
}

void velocity_pattern(const Csr& G, const uint8_t* dir, uint8_t* cv, VPatternOut& out,
                      hipStream_t s, Arena& ar, int lds_max) {
  const int64_t n = G.nrows;
  int* err = ar.alloc<int>(1);
  HIP_OK(hipMemsetAsync(err, 0, sizeof(int), s));
  uint8_t* cov = ar.alloc<uint8_t>(n);
  int32_t* vcnt = ar.alloc<int32_t>(n);
  int32_t* vbuf = ar.alloc<int32_t>((size_t)n * VCAP);
  int32_t* vis = ar.alloc<int32_t>(n);
  HIP_OK(hipMemsetAsync(cov, 0, n, s));
  HIP_OK(hipMemsetAsync(vcnt, 0, sizeof(int32_t) * n, s));
  HIP_OK(hipMemsetAsync(vis, 0xFF, sizeof(int32_t) * n, s));
  // initial C^(v) list; its size, the longest graph row and the index
  // bandwidth in one read-back
  int64_t* incl = ar.alloc<int64_t>(n + 1);
  unsigned long long* mx2 = ar.alloc<unsigned long long>(2);
  int64_t* q = ar.alloc<int64_t>(5);
  if (n) k_flags_u8<<<nblocks(n, 256), 256, 0, s>>>(cv, n, incl);
  scan_inclusive(incl, n, s, ar);
  max_row_len_dev(G.rowptr, n, mx2, s);
  index_bandwidth_dev(G.rowptr, G.col, n, mx2 + 1, s);
  k_gather_scalars<<<1, 64, 0, s>>>(n ? incl + n - 1 : nullptr, nullptr, mx2, mx2 + 1, nullptr, q);
  int64_t hq[5];
  HIP_OK(hipMemcpyAsync(hq, q, sizeof(hq), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t n0 = hq[0];
  int32_t* src0 = ar.alloc<int32_t>(n0);
  if (n) k_compact_u8<<<nblocks(n, 256), 256, 0, s>>>(incl, cv, n, src0, nullptr);
  if (n0) k_vbfs<<<nblocks(n0, VB_WAVES), 64 * VB_WAVES, 0, s>>>(G.rowptr, G.col, src0, n0, dir,
                                                                  cov, vcnt, vbuf, err);
  // extra points in ascending order
  const int64_t maxdeg = hq[2];
  int deg_cap = 1;
  while (deg_cap < maxdeg && deg_cap < 1024) deg_cap <<= 1;
  int32_t* extra = ar.alloc<int32_t>(n);
  int32_t* nextra = ar.alloc<int32_t>(1);
  int ballcap = 8192;
  if (ballcap * 4 + 64 > lds_max) ballcap = (lds_max - 64) / 4;
  // visited bitmap over the ball's index window when it fits beside the list
  const int64_t bw = hq[3];
  const int64_t words = (6 * bw + 1 + 31) / 32;
  const int nwin = (int64_t)ballcap * 4 + words * 4 + 64 <= lds_max ? (int)words : 0;
  const size_t lds = (size_t)ballcap * 4 + (size_t)nwin * 4;
  allow_lds((const void*)k_vextras);
  prof::Scope ps(s, EMIN_PROF_VPAT, 0.0);
  k_vextras<<<1, 1024, lds, s>>>(G.rowptr, G.col, n, dir, cv, cov, vis, extra, nextra, ballcap,
                                  deg_cap, bw, nwin, err);
  HIP_OK(hipGetLastError());
  out.n_extra = d2h(nextra, s);
  if (out.n_extra)
    k_vbfs<<<nblocks(out.n_extra, VB_WAVES), 64 * VB_WAVES, 0, s>>>(
        G.rowptr, G.col, extra, out.n_extra, dir, cov, vcnt, vbuf, err);
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
  HIP_OK(hipMemcpyAsync(hc, q, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (hc[4]) throw Error(EMIN_ERR_CAPACITY, "velocity pattern: row or ball capacity");
  out.n_c = hc[0];
  out.N.nnz = hc[1];
  out.N.ncols = out.n_c;
  out.cid = ar.alloc<int32_t>(n);
  out.clist = ar.alloc<int32_t>(out.n_c);
  if (n) k_compact_u8<<<nblocks(n, 256), 256, 0, s>>>(incl, cv, n, out.clist, out.cid);
  out.N.col = ar.alloc<int32_t>(out.N.nnz);
  if (n)
    k_v_fill<<<nblocks(n, 256), 256, 0, s>>>(cv, dir, vcnt, vbuf, out.cid, n, out.N.rowptr,
                                              out.N.col);
}

}  // namespace emin
