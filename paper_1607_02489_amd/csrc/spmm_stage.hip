// Masked product Q = mask_N(M Z) with LDS-staged rows of Z (sec. 4.3).
//
// A block owns SR consecutive rows i.  Every Z row k that those rows' M
// entries reach is copied once into LDS: the union of the k's is a handful of
// runs of consecutive indices (one per neighbouring line of the mesh in a
// lexicographic ordering), and since pattern rows are stored back to back, a
// run of k's is one contiguous range of Z's values -- a coalesced stream.
// The block's slice of M (values, intersection maps) is contiguous too.  All
// the irregular work -- finding Z(k, j) for slot j of row i -- then reads
// LDS, and HBM sees only coalesced loads and stores.
//
// Per output entry (i, slot s) the sum runs over M's row i in ascending k,
// one fused multiply-add per matching entry, exactly as the gathering kernel
// does, so both give the same bits.  The plan (which blocks fit, their runs,
// each M entry's LDS offset) is built once per pattern.
#include "emin_cg.h"
#include "prof.h"

#include <hip/hip_ext.h>

namespace emin {

namespace {

constexpr int ST_BS = 128;            // threads per block
constexpr int ST_WBITS = 32768;       // plan: widest k window (bits of the LDS bitmap)

__device__ __forceinline__ int block_excl_scan(int v, int* tmp) {
  // exclusive scan over the block (ST_BS threads); tmp holds ST_BS/64 + 1
  // ints, and its total stays in tmp[ST_BS/64] until the next call
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
    for (int k = 0; k < ST_BS / 64; k++) {
      const int t = tmp[k];
      tmp[k] = a;
      a += t;
    }
    tmp[ST_BS / 64] = a;
  }
  __syncthreads();
  const int r = tmp[w] + x - v;
  return r;
}

// Plan of one block of SR rows.  Pass 0 decides whether the block is staged
// (every row map-eligible, at most EMAX M entries, a k window of at most
// ST_WBITS, at most VCAP staged values and RCAP runs) and counts its runs and
// the M / pattern entries it covers; pass 1 (staged blocks only) writes the
// runs and every M entry's LDS offset.
template <int PASS>
__global__ __launch_bounds__(ST_BS) void k_stage_plan(StageDims D, const int64_t* mrp,
                                                      const int32_t* mcol, const int64_t* nrp,
                                                      const int32_t* kofs, const uint8_t* elig,
                                                      int64_t n, uint8_t* flag, int32_t* nruns,
                                                      const int64_t* roff, int32_t* rg,
                                                      int32_t* rl, int32_t* rn, int32_t* lofs,
                                                      unsigned long long* cnt) {
  __shared__ uint32_t bits[ST_WBITS / 32];
  __shared__ int32_t wpre[ST_WBITS / 32];
  __shared__ int tmp[ST_BS / 64 + 1];
  __shared__ int s_ok;
  __shared__ int s_kmin, s_kmax;
  extern __shared__ int32_t dyn[];   // u list (EMAX), offsets (EMAX + 1)
  int32_t* s_u = dyn;
  int32_t* s_off = dyn + D.emax;
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * D.sr;
  const int64_t r1 = r0 + D.sr < n ? r0 + D.sr : n;
  if (PASS == 1 && !flag[b]) return;
  if (threadIdx.x == 0) {
    s_ok = 1;
    s_kmin = INT32_MAX;
    s_kmax = -1;
  }
  __syncthreads();
  const int64_t e0 = mrp[r0], e1 = mrp[r1];
  const int64_t K = e1 - e0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += ST_BS)
    if (!elig[i]) s_ok = 0;
  if (K > D.emax) s_ok = 0;
  __syncthreads();
  if (!s_ok) {
    if (PASS == 0 && threadIdx.x == 0) {
      flag[b] = 0;
      nruns[b] = 0;
    }
    return;
  }
  int kmn = INT32_MAX, kmx = -1;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += ST_BS) {
    const int32_t k = mcol[e];
    kmn = k < kmn ? k : kmn;
    kmx = k > kmx ? k : kmx;
  }
  if (kmx >= 0) {
    atomicMin(&s_kmin, kmn);
    atomicMax(&s_kmax, kmx);
  }
  for (int t = threadIdx.x; t < ST_WBITS / 32; t += ST_BS) bits[t] = 0u;
  __syncthreads();
  const int kmin = s_kmin, kmax = s_kmax;
  const int width = kmax >= kmin ? kmax - kmin + 1 : 0;
  if (width > ST_WBITS) {
    if (PASS == 0 && threadIdx.x == 0) {
      flag[b] = 0;
      nruns[b] = 0;
    }
    return;
  }
  for (int64_t e = e0 + threadIdx.x; e < e1; e += ST_BS) {
    const int o = mcol[e] - kmin;
    atomicOr(&bits[o >> 5], 1u << (o & 31));
  }
  __syncthreads();
  // rank of every bitmap word: per thread a contiguous slice of words
  const int nw = (width + 31) >> 5;
  const int per = (nw + ST_BS - 1) / ST_BS;
  const int w0 = threadIdx.x * per, w1 = w0 + per < nw ? w0 + per : nw;
  int c = 0;
  for (int w = w0; w < w1; w++) c += __popc(bits[w]);
  int base = block_excl_scan(c, tmp);
  const int U = tmp[ST_BS / 64];
  for (int w = w0; w < w1; w++) {
    wpre[w] = base;
    uint32_t m = bits[w];
    while (m) {
      const int bt = __ffs(m) - 1;
      m &= m - 1u;
      s_u[base++] = kmin + 32 * w + bt;
    }
  }
  __syncthreads();
  // staged values: pattern row lengths of the union, prefix offsets
  const int per_u = (U + ST_BS - 1) / ST_BS;
  const int u0 = threadIdx.x * per_u, u1 = u0 + per_u < U ? u0 + per_u : U;
  int lsum = 0, rs = 0;
  for (int u = u0; u < u1; u++) {
    const int32_t k = s_u[u];
    lsum += (int)(nrp[k + 1] - nrp[k]);
    rs += (u == 0 || s_u[u - 1] != k - 1) ? 1 : 0;
  }
  int obase = block_excl_scan(lsum, tmp);
  const int V = tmp[ST_BS / 64];
  int rbase = block_excl_scan(rs, tmp);
  const int NR = tmp[ST_BS / 64];
  if (V > D.vcap || NR > D.rcap) {
    if (PASS == 0 && threadIdx.x == 0) {
      flag[b] = 0;
      nruns[b] = 0;
    }
    return;
  }
  if (PASS == 0) {
    if (threadIdx.x == 0) {
      flag[b] = 1;
      nruns[b] = NR;
      atomicAdd(cnt + 0, (unsigned long long)(r1 - r0));
      atomicAdd(cnt + 1, (unsigned long long)K);
      atomicAdd(cnt + 2, (unsigned long long)(nrp[r1] - nrp[r0]));
      atomicAdd(cnt + 3, 1ull);
    }
    return;
  }
  for (int u = u0; u < u1; u++) {
    s_off[u] = obase;
    obase += (int)(nrp[s_u[u] + 1] - nrp[s_u[u]]);
  }
  if (threadIdx.x == 0) s_off[U] = V;
  __syncthreads();
  // runs: a start where k does not continue the previous union entry; its
  // length runs to the next start
  const int64_t ro = roff[b];
  for (int u = u0; u < u1; u++) {
    const int32_t k = s_u[u];
    if (u == 0 || s_u[u - 1] != k - 1) {
      int v = u + 1;
      while (v < U && s_u[v] == s_u[v - 1] + 1) v++;
      rg[ro + rbase] = (int32_t)nrp[k];
      rl[ro + rbase] = s_off[u];
      rn[ro + rbase] = s_off[v] - s_off[u];
      rbase++;
    }
  }
  // every M entry: its row k's LDS start plus the map's base shift
  for (int64_t e = e0 + threadIdx.x; e < e1; e += ST_BS) {
    const int32_t k = mcol[e];
    const int o = k - kmin;
    const int u = wpre[o >> 5] + __popc(bits[o >> 5] & ((1u << (o & 31)) - 1u));
    lofs[e] = s_off[u] + (int32_t)((int64_t)kofs[e] - nrp[k]);
  }
}

__global__ void k_stage_list(const uint8_t* flag, int64_t nb, const int64_t* incl, int32_t* list,
                             int sr, int64_t n, uint8_t* row_staged) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const bool f = flag[b] != 0;
  if (f) list[incl[b] - 1] = (int32_t)b;
  const int64_t r0 = b * sr;
  for (int64_t i = r0; i < r0 + sr && i < n; i++) row_staged[i] = f ? 1 : 0;
}

__global__ void k_i32_to_i64(const int32_t* a, int64_t* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_flag_to_i64(const uint8_t* a, int64_t* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] ? 1 : 0;
}

}  // namespace

// LDS bytes of the product kernel for one plan
static size_t stage_smem(const StageDims& D, int np, size_t tm, size_t tx) {
  size_t b = 0;
  b += (size_t)3 * D.rcap * 4;                       // runs
  b += (size_t)(D.sr + 1) * 4 * 2;                   // local row pointers of M and N
  b = (b + 15) & ~size_t(15);
  b += (size_t)D.vcap * tx;                          // staged Z
  b = (b + 15) & ~size_t(15);
  b += (size_t)D.emax * (tm + 4 + 4 * (size_t)np);   // M values, LDS offsets, map words
  return (b + 15) & ~size_t(15);
}

void stage_plan(EminWork& w, const Csr& M, const int64_t* nrp, const uint8_t* elig, hipStream_t s,
                Arena& ar) {
  StagePlan& P = w.stage;
  P = StagePlan{};
  const int64_t n = w.n;
  if (n == 0 || w.nnz == 0) return;
  StageDims D;
  D.sr = 16;
  D.emax = 640;
  D.rcap = 64;
  D.vcap = 3072;
  D.np = w.nplanes;
  const int64_t nb = (n + D.sr - 1) / D.sr;
  if (nb >= INT32_MAX) return;
  uint8_t* flag = ar.alloc<uint8_t>(nb);
  int32_t* nr = ar.alloc<int32_t>(nb);
  unsigned long long* cnt = ar.alloc<unsigned long long>(4);
  HIP_OK(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), s));
  const size_t dyn = (size_t)(2 * D.emax + 1) * 4;
  k_stage_plan<0><<<(unsigned)nb, ST_BS, dyn, s>>>(D, M.rowptr, M.col, nrp, w.kofs, elig, n, flag,
                                                   nr, nullptr, nullptr, nullptr, nullptr,
                                                   nullptr, cnt);
  // run offsets and the list of staged blocks
  int64_t* roff = ar.alloc<int64_t>(nb + 1);
  HIP_OK(hipMemsetAsync(roff, 0, sizeof(int64_t), s));
  k_i32_to_i64<<<nblocks(nb, 256), 256, 0, s>>>(nr, roff + 1, nb);
  scan_inclusive(roff + 1, nb, s, ar);
  int64_t* fl = ar.alloc<int64_t>(nb);
  k_flag_to_i64<<<nblocks(nb, 256), 256, 0, s>>>(flag, fl, nb);
  scan_inclusive(fl, nb, s, ar);
  unsigned long long hc[4];
  int64_t tot_runs = 0;
  HIP_OK(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&tot_runs, roff + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t nst = (int64_t)hc[3];
  if (nst == 0) return;
  int32_t* rg = ar.alloc<int32_t>(tot_runs);
  int32_t* rl = ar.alloc<int32_t>(tot_runs);
  int32_t* rn = ar.alloc<int32_t>(tot_runs);
  int32_t* lofs = ar.alloc<int32_t>(M.nnz);
  k_stage_plan<1><<<(unsigned)nb, ST_BS, dyn, s>>>(D, M.rowptr, M.col, nrp, w.kofs, elig, n, flag,
                                                   nr, roff, rg, rl, rn, lofs, nullptr);
  int32_t* list = ar.alloc<int32_t>(nst);
  uint8_t* rs = ar.alloc<uint8_t>(n);
  k_stage_list<<<nblocks(nb, 256), 256, 0, s>>>(flag, nb, fl, list, D.sr, n, rs);
  P.dims = D;
  P.nblk = nst;
  P.blocks = list;
  P.roff = roff;
  P.rg = rg;
  P.rl = rl;
  P.rn = rn;
  P.lofs = lofs;
  P.row_staged = rs;
  P.rows = (int64_t)hc[0];
  P.m_entries = (int64_t)hc[1];
  P.p_entries = (int64_t)hc[2];
}

// The product on the staged blocks.  Phases: the block's runs and row
// pointers to LDS; Z's runs and M's slice to LDS (coalesced); one output
// entry per thread at a time (the row by binary search over the local row
// pointers), summing over the row's M entries from LDS; Y stored coalesced;
// with D, each row's <D, Y> summed in slot order.
template <class TM, class TX, class TY>
__global__ __launch_bounds__(ST_BS) void k_spmm_stage(StageArgs A, const int64_t* mrp,
                                                      const TM* mval, const uint32_t* nib,
                                                      int64_t nnzm, const int64_t* nrp,
                                                      const TX* X, TY* Y, const double* Dv,
                                                      double* rowdot) {
  extern __shared__ __align__(16) unsigned char smem[];
  const StageDims& D = A.dims;
  int32_t* s_rg = reinterpret_cast<int32_t*>(smem);
  int32_t* s_rl = s_rg + D.rcap;
  int32_t* s_rn = s_rl + D.rcap;
  int32_t* s_mr = s_rn + D.rcap;          // local M row pointers (sr + 1)
  int32_t* s_nr = s_mr + D.sr + 1;        // local N row pointers (sr + 1)
  size_t off = ((size_t)(3 * D.rcap + 2 * (D.sr + 1)) * 4 + 15) & ~size_t(15);
  TX* s_z = reinterpret_cast<TX*>(smem + off);
  off = (off + (size_t)D.vcap * sizeof(TX) + 15) & ~size_t(15);
  TM* s_m = reinterpret_cast<TM*>(smem + off);
  int32_t* s_lo = reinterpret_cast<int32_t*>(s_m + D.emax);
  uint32_t* s_w = reinterpret_cast<uint32_t*>(s_lo + D.emax);   // [np][emax]

  const int64_t b = A.blocks[xcd_block(blockIdx.x, gridDim.x)];
  const int64_t n = A.n;
  const int64_t r0 = b * D.sr;
  const int64_t r1 = r0 + D.sr < n ? r0 + D.sr : n;
  const int nrows = (int)(r1 - r0);
  const int64_t ro = A.roff[b];
  const int nr = (int)(A.roff[b + 1] - ro);
  const int t = threadIdx.x;
  const int64_t e0 = mrp[r0], p0 = nrp[r0];
  for (int q = t; q < nr; q += ST_BS) {
    s_rg[q] = A.rg[ro + q];
    s_rl[q] = A.rl[ro + q];
    s_rn[q] = A.rn[ro + q];
  }
  for (int q = t; q <= nrows; q += ST_BS) {
    s_mr[q] = (int32_t)(mrp[r0 + q] - e0);
    s_nr[q] = (int32_t)(nrp[r0 + q] - p0);
  }
  __syncthreads();
  // Z's runs: each wave copies whole runs, lanes along the run
  {
    const int lane = t & 63, wv = t >> 6;
    for (int q = wv; q < nr; q += ST_BS / 64) {
      const TX* src = X + s_rg[q];
      TX* dst = s_z + s_rl[q];
      const int len = s_rn[q];
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
  }
  // M's slice: values, LDS offsets, map words
  const int K = s_mr[nrows];
  for (int q = t; q < K; q += ST_BS) {
    s_m[q] = mval[e0 + q];
    s_lo[q] = A.lofs[e0 + q];
    for (int p = 0; p < D.np; p++) s_w[p * D.emax + q] = nib[(int64_t)p * nnzm + e0 + q];
  }
  __syncthreads();
  const int NE = s_nr[nrows];
  constexpr int EPT = 4;                  // output entries per thread (sr * 32 / ST_BS)
  TM acc[EPT];
  int rowi[EPT];
#pragma unroll
  for (int j = 0; j < EPT; j++) {
    const int p = t + j * ST_BS;
    acc[j] = TM(0);
    rowi[j] = -1;
    if (p < NE) {
      int lo = 0, hi = nrows - 1;          // last row whose start <= p
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_nr[mid] <= p) lo = mid; else hi = mid - 1;
      }
      const int sl = p - s_nr[lo];
      rowi[j] = lo;
      const int sh = 4 * (sl & 7);
      const uint32_t* wp = s_w + (sl >> 3) * D.emax;
      TM a = TM(0);
      for (int e = s_mr[lo]; e < s_mr[lo + 1]; e++) {
        const uint32_t f = (wp[e] >> sh) & 0xFu;
        if (f != 0xFu) a = fma(s_m[e], (TM)s_z[s_lo[e] + sl + (int)f], a);
      }
      acc[j] = a;
      Y[p0 + p] = (TY)a;
    }
  }
  if (!Dv) return;
  __syncthreads();                        // every thread is done with s_z
  double* s_pr = reinterpret_cast<double*>(s_z);
#pragma unroll
  for (int j = 0; j < EPT; j++) {
    const int p = t + j * ST_BS;
    if (p < NE) s_pr[p] = Dv[p0 + p] * (double)acc[j];
  }
  __syncthreads();
  for (int r = t; r < nrows; r += ST_BS) {
    double sum = 0.0;
    for (int p = s_nr[r]; p < s_nr[r + 1]; p++) sum = sum + s_pr[p];
    rowdot[r0 + r] = sum;
  }
}

template <class TM, class TX, class TY>
void spmm_stage(const EminWork& w, const int64_t* mrp, const TM* mval, const int64_t* nrp,
                const TX* X, TY* Y, const double* Dv, double bytes, hipStream_t s) {
  const StagePlan& P = w.stage;
  if (P.nblk == 0) return;
  StageArgs A;
  A.dims = P.dims;
  A.blocks = P.blocks;
  A.roff = P.roff;
  A.rg = P.rg;
  A.rl = P.rl;
  A.rn = P.rn;
  A.lofs = P.lofs;
  A.n = w.n;
  const size_t lds = stage_smem(P.dims, P.dims.np, sizeof(TM), sizeof(TX));
  allow_lds((const void*)k_spmm_stage<TM, TX, TY>);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof::begin_launch(s, EMIN_PROF_SPMM, bytes, 0.0, &e0, &e1)) {
    hipExtLaunchKernelGGL(k_spmm_stage<TM, TX, TY>, dim3((unsigned)P.nblk), dim3(ST_BS), lds, s,
                          e0, e1, 0, A, mrp, mval, (const uint32_t*)w.nib, w.nnzm, nrp, X, Y, Dv,
                          w.rowdot);
    HIP_OK(hipGetLastError());
  } else {
    k_spmm_stage<TM, TX, TY><<<(unsigned)P.nblk, ST_BS, lds, s>>>(A, mrp, mval, w.nib, w.nnzm, nrp,
                                                                 X, Y, Dv, w.rowdot);
  }
}

template void spmm_stage<double, double, double>(const EminWork&, const int64_t*, const double*,
                                                 const int64_t*, const double*, double*,
                                                 const double*, double, hipStream_t);
template void spmm_stage<float, float, float>(const EminWork&, const int64_t*, const float*,
                                              const int64_t*, const float*, float*, const double*,
                                              double, hipStream_t);

}  // namespace emin
