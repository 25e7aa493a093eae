// Sparse building blocks: scans, transposes, the ordered row-wise SpGEMM,
// and the drop/lump filter of eq. (e:filtering) with its symmetrisation.
#include "common.h"
#include "prof.h"

namespace emin {

// ---------------------------------------------------------------------------
// scan
// ---------------------------------------------------------------------------
constexpr int SCAN_BS = 256;
constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IT;

__device__ int64_t block_exclusive(int64_t v, int64_t* lds, int64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int k = 0; k < SCAN_BS / 64; k++) {
    if (k < w) off += lds[k];
    tot += lds[k];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void k_tile_sums(const int64_t* a, int64_t n, int64_t* bsum) {
  __shared__ int64_t lds[SCAN_BS / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
  int64_t s = 0;
  for (int j = 0; j < SCAN_IT; j++)
    if (base + j < n) s += a[base + j];
  int64_t tot;
  block_exclusive(s, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_tile_scan(int64_t* a, int64_t n, const int64_t* bincl) {
  __shared__ int64_t lds[SCAN_BS / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
  int64_t v[SCAN_IT];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IT; j++) {
    v[j] = (base + j < n) ? a[base + j] : 0;
    s += v[j];
  }
  int64_t tot;
  int64_t off = block_exclusive(s, lds, &tot);
  if (bincl && blockIdx.x > 0) off += bincl[blockIdx.x - 1];
#pragma unroll
  for (int j = 0; j < SCAN_IT; j++) {
    off += v[j];
    if (base + j < n) a[base + j] = off;
  }
}

void scan_inclusive(int64_t* a, int64_t n, hipStream_t s, Arena& ar) {
  if (n <= 0) return;
  unsigned nb = nblocks(n, SCAN_TILE);
  if (nb == 1) {
    k_tile_scan<<<1, SCAN_BS, 0, s>>>(a, n, nullptr);
    return;
  }
  int64_t* bs = ar.alloc<int64_t>(nb);
  k_tile_sums<<<nb, SCAN_BS, 0, s>>>(a, n, bs);
  scan_inclusive(bs, nb, s, ar);
  k_tile_scan<<<nb, SCAN_BS, 0, s>>>(a, n, bs);
}

// Index bandwidth of a graph, max |i - j| over its edges: every vertex within
// distance d of v lies in [v - d bw, v + d bw].
__global__ void k_bandwidth(const int64_t* grp, const int32_t* gcol, int64_t n,
                            unsigned long long* bw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long m = 0ull;
  if (i < n)
    for (int64_t e = grp[i]; e < grp[i + 1]; e++) {
      const int64_t d = (int64_t)gcol[e] - i;
      const unsigned long long a = (unsigned long long)(d < 0 ? -d : d);
      m = a > m ? a : m;
    }
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long t = __shfl_xor(m, o, 64);
    m = t > m ? t : m;
  }
  if ((threadIdx.x & 63) == 0 && m > __hip_atomic_load(bw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(bw, m);
}

void index_bandwidth_dev(const int64_t* rp, const int32_t* col, int64_t n,
                         unsigned long long* out, hipStream_t s) {
  HIP_OK(hipMemsetAsync(out, 0, sizeof(unsigned long long), s));
  if (n > 0) k_bandwidth<<<nblocks(n, 256), 256, 0, s>>>(rp, col, n, out);
}

int64_t index_bandwidth(const int64_t* rp, const int32_t* col, int64_t n, hipStream_t s,
                        Arena& ar) {
  if (n <= 0) return 0;
  unsigned long long* bw = ar.alloc<unsigned long long>(1);
  index_bandwidth_dev(rp, col, n, bw, s);
  return (int64_t)d2h(bw, s);
}

int64_t rowptr_from_counts(int64_t* rowptr, int64_t n, hipStream_t s, Arena& ar) {
  HIP_OK(hipMemsetAsync(rowptr, 0, sizeof(int64_t), s));
  scan_inclusive(rowptr + 1, n, s, ar);
  return d2h(rowptr + n, s);
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Row kernels with G lanes per row (G a power of two, at most 64, so a group
// never spans two waves): loads of a row are coalesced and its entries are
// processed in parallel.  Control flow is uniform within a group.
// ---------------------------------------------------------------------------
static int lanes_for(const CsrView& A) {
  const double avg = A.nrows ? (double)A.nnz / (double)A.nrows : 1.0;
  int g = 4;
  while (g < 64 && g < avg) g <<= 1;
  return g;
}


#define ROWS_DISPATCH(g, KERNEL, n, s, ...)                                              \
  do {                                                                                   \
    switch (g) {                                                                         \
      case 4: KERNEL<4><<<nblocks(n, 64), 256, 0, s>>>(__VA_ARGS__); break;              \
      case 8: KERNEL<8><<<nblocks(n, 32), 256, 0, s>>>(__VA_ARGS__); break;              \
      case 16: KERNEL<16><<<nblocks(n, 16), 256, 0, s>>>(__VA_ARGS__); break;            \
      case 32: KERNEL<32><<<nblocks(n, 8), 256, 0, s>>>(__VA_ARGS__); break;             \
      default: KERNEL<64><<<nblocks(n, 4), 256, 0, s>>>(__VA_ARGS__); break;             \
    }                                                                                    \
  } while (0)

template <int G>
__global__ __launch_bounds__(256) void k_validate_g(const int64_t* rp, const int32_t* col,
                                                   const double* val, int64_t n, int64_t ncols,
                                                   int64_t nnz, int* derr) {
  const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (i >= n) return;
  const int64_t a = rp[i], b = rp[i + 1];
  if (a < 0 || b < a || b > nnz) {
    if (lane == 0) atomicOr(derr, DERR_PATTERN);
    return;
  }
  bool badp = false, badv = false;
  for (int64_t e = a + lane; e < b; e += G) {
    const int32_t c = col[e];
    const int32_t prev = e > a ? col[e - 1] : -1;
    if (c <= prev || c >= ncols) badp = true;
    if (val && !isfinite(val[e])) badv = true;
  }
  if (badp) atomicOr(derr, DERR_PATTERN);
  if (badv) atomicOr(derr, DERR_VALUE);
}

// eq. (e:filtering), squared form, per entry; the row count adds the diagonal.
// dir (optional): the Dirichlet flags of the rows, from the same pass (a row
// is Dirichlet when no off-diagonal value is nonzero)
template <int G>
__global__ __launch_bounds__(256) void k_filter_count_g(const int64_t* rp, const int32_t* col,
                                                       const double* val, int64_t n, double t2,
                                                       const double* d, uint8_t* keep,
                                                       int64_t* cnt, uint8_t* dir) {
  const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (i >= n) return;
  const double di = d[i];
  int64_t c = 1;
  bool nz = false;
  for (int64_t e0 = rp[i]; e0 < rp[i + 1]; e0 += G) {
    const int64_t e = e0 + lane;
    bool kept_off = false;
    if (e < rp[i + 1]) {
      const int32_t j = col[e];
      uint8_t k = 1;
      if (j != i) {
        const double v = val[e];
        const double lhs = v * v;
        const double rhs = t2 * fabs(di * d[j]);
        k = lhs > rhs;
        kept_off = k;
        if (v != 0.0) nz = true;
      }
      keep[e] = k;
    }
    c += __popcll(group_ballot<G>(kept_off));
  }
  const uint64_t m = group_ballot<G>(nz);
  if (lane == 0) {
    cnt[i + 1] = c;
    if (dir) dir[i] = m ? 0 : 1;
  }
}

// Filtered row: kept off-diagonals in column order with the diagonal at its
// sorted place; the diagonal is a_ii plus the dropped entries added one by
// one in ascending column order (the same sums, in the same order, as a
// sequential pass over the row).
template <int G>
__global__ __launch_bounds__(256) void k_filter_fill_g(const int64_t* rp, const int32_t* col,
                                                      const double* val, int64_t n,
                                                      const uint8_t* keep, const double* d,
                                                      const int64_t* orp, int32_t* ocol,
                                                      double* oval) {
  const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (i >= n) return;
  const int64_t a = rp[i], b = rp[i + 1], base = orp[i];
  const uint64_t below = (1ull << lane) - 1ull;
  double lump = d[i];
  int64_t kept = 0, kept_lt = 0;
  for (int64_t e0 = a; e0 < b; e0 += G) {
    const int64_t e = e0 + lane;
    const bool ok = e < b;
    const int32_t j = ok ? col[e] : (int32_t)i;
    const double v = ok ? val[e] : 0.0;
    const bool k = ok && j != i && keep[e];
    const bool dropped = ok && j != i && !keep[e];
    uint64_t md = group_ballot<G>(dropped);
    if constexpr (G == 64) {
      // the group is the wave: t is uniform, and a lane read through the
      // scalar unit is far shorter than a shuffle on this serial chain
      const int64_t vb = __double_as_longlong(v);
      const int32_t vlo = (int32_t)(vb & 0xffffffffll), vhi = (int32_t)(vb >> 32);
      while (md) {
        const int t = __builtin_ctzll(md);
        md &= md - 1ull;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(vlo, t);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(vhi, t);
        lump = lump + __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
      }
    } else {
      while (md) {
        const int t = __builtin_ctzll(md);
        md &= md - 1ull;
        lump = lump + __shfl(v, t, G);
      }
    }
    const uint64_t mk = group_ballot<G>(k);
    if (k) {
      const int64_t p = base + kept + __popcll(mk & below) + (j > i ? 1 : 0);
      if (ocol) ocol[p] = j;
      oval[p] = v;
    }
    kept += __popcll(mk);
    kept_lt += __popcll(group_ballot<G>(k && j < i));
  }
  if (lane == 0) {
    if (ocol) ocol[base + kept_lt] = (int32_t)i;
    oval[base + kept_lt] = lump;
  }
}


void validate_csr(const CsrView& A, bool values, int* derr, hipStream_t s) {
  if (A.nrows == 0) return;
  ROWS_DISPATCH(lanes_for(A), k_validate_g, A.nrows, s, A.rowptr, A.col,
                values ? A.val : nullptr, A.nrows, A.ncols, A.nnz, derr);
}

// ---------------------------------------------------------------------------
// transpose
// ---------------------------------------------------------------------------
__global__ void k_widen_u32(const uint32_t* a, int64_t n, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i];
}

__global__ void k_narrow_i64(const int64_t* a, int64_t n, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint32_t)a[i];
}


// Restores ascending order inside each row of the transpose (the atomic fill
// leaves it arbitrary; keys are distinct within a row).  Rows are binned by
// length without a host round trip (device-side lists), then
//  - rows of at most 64 entries: G lanes per row, each lane ranks its key
//    against the row's others through wave shuffles and writes it in place;
//  - longer rows: one block per row, bitonic sort of the padded row in LDS
//    (rows beyond the largest LDS size: the same network in global memory).
// The network is the variant in which every comparator puts the smaller key
// at the lower index (the first stage of each merge compares mirrored
// positions), so padding keys (+inf) beyond the row's end never move into it.
// Every bin kernel walks its list grid-stride and reads the list length on
// the device, so the launches do not wait for the classification.
constexpr int SORT_NBIN = 9;   // G = 4, 8, 16, 32, 64; P = 512, 2048, 16384; longer
constexpr int SORT_PMAX = 16384;

__device__ __forceinline__ int sort_bin(int64_t L) {
  if (L <= 4) return 0;
  if (L <= 8) return 1;
  if (L <= 16) return 2;
  if (L <= 32) return 3;
  if (L <= 64) return 4;
  if (L <= 512) return 5;
  if (L <= 2048) return 6;
  if (L <= SORT_PMAX) return 7;
  return 8;
}

// one global atomic per bin per block (LDS counters first)
__global__ __launch_bounds__(1024) void k_sort_classify(const int64_t* rp, int64_t n,
                                                       int32_t* lists, int32_t* counts) {
  __shared__ int lcnt[SORT_NBIN], lbase[SORT_NBIN];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x < SORT_NBIN) lcnt[threadIdx.x] = 0;
  __syncthreads();
  int b = -1;
  if (i < n) {
    const int64_t L = rp[i + 1] - rp[i];
    if (L > 1) b = sort_bin(L);
  }
  const int lpos = b >= 0 ? atomicAdd(&lcnt[b], 1) : 0;
  __syncthreads();
  if (threadIdx.x < SORT_NBIN && lcnt[threadIdx.x])
    lbase[threadIdx.x] = atomicAdd(&counts[threadIdx.x], lcnt[threadIdx.x]);
  __syncthreads();
  if (b >= 0) lists[(int64_t)b * n + lbase[b] + lpos] = (int32_t)i;
}

template <int G>
__global__ __launch_bounds__(256) void k_sort_group(const int64_t* rp, const int32_t* rows,
                                                    const int32_t* count, int32_t* key,
                                                    int32_t* src) {
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t nr = *count;
  for (int64_t r0 = (int64_t)blockIdx.x * NG; r0 < nr; r0 += (int64_t)gridDim.x * NG) {
    const int64_t r = r0 + g;
    int64_t a = 0;
    int L = 0;
    if (r < nr) {
      const int32_t i = rows[r];
      a = rp[i];
      L = (int)(rp[i + 1] - a);
    }
    const bool mine = lane < L;
    const int32_t k = mine ? key[a + lane] : INT32_MAX;
    const int32_t sv = mine ? src[a + lane] : 0;
    int rank = 0;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int32_t ku = __shfl(k, u, G);
      rank += (ku < k) ? 1 : 0;
    }
    if (mine) {
      key[a + rank] = k;
      src[a + rank] = sv;
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_sort_block(const int64_t* rp, const int32_t* rows,
                                                    const int32_t* count, int32_t* key,
                                                    int32_t* src) {
  extern __shared__ int32_t sb[];
  int32_t* tk = sb;
  int32_t* ts = sb + P;
  const int64_t nr = *count;
  for (int64_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const int32_t i = rows[r];
    const int64_t a = rp[i];
    const int L = (int)(rp[i + 1] - a);
    for (int t = threadIdx.x; t < P; t += 256) {
      tk[t] = t < L ? key[a + t] : INT32_MAX;
      ts[t] = t < L ? src[a + t] : 0;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < P / 2; t += 256) {
          const int lo = 2 * t - (t & (j - 1));   // index with bit j clear
          const int hi = j == (k >> 1) ? (lo | (k - 1)) - (lo & (k - 1)) : lo + j;
          const int32_t x = tk[lo], y = tk[hi];
          if (x > y) {
            tk[lo] = y;
            tk[hi] = x;
            const int32_t sx = ts[lo];
            ts[lo] = ts[hi];
            ts[hi] = sx;
          }
        }
        __syncthreads();
      }
    }
    for (int t = threadIdx.x; t < L; t += 256) {
      key[a + t] = tk[t];
      src[a + t] = ts[t];
    }
    __syncthreads();
  }
}

// rows longer than the LDS network: the same comparators on the row in place
__global__ __launch_bounds__(256) void k_sort_global(const int64_t* rp, const int32_t* rows,
                                                     const int32_t* count, int32_t* key,
                                                     int32_t* src) {
  const int64_t nr = *count;
  for (int64_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const int32_t i = rows[r];
    int32_t* tk = key + rp[i];
    int32_t* ts = src + rp[i];
    const int64_t L = rp[i + 1] - rp[i];
    int64_t P = 1;
    while (P < L) P <<= 1;
    for (int64_t k = 2; k <= P; k <<= 1) {
      for (int64_t j = k >> 1; j > 0; j >>= 1) {
        for (int64_t t = threadIdx.x; t < P / 2; t += 256) {
          const int64_t lo = 2 * t - (t & (j - 1));
          const int64_t hi = j == (k >> 1) ? (lo | (k - 1)) - (lo & (k - 1)) : lo + j;
          if (hi < L) {
            const int32_t x = tk[lo], y = tk[hi];
            if (x > y) {
              tk[lo] = y;
              tk[hi] = x;
              const int32_t sx = ts[lo];
              ts[lo] = ts[hi];
              ts[hi] = sx;
            }
          }
        }
        __syncthreads();
      }
    }
  }
}

void sort_rows(const int64_t* rp, int64_t n, int32_t* key, int32_t* src, hipStream_t s,
               Arena& ar) {
  if (n == 0) return;
  int32_t* lists = ar.alloc<int32_t>((size_t)SORT_NBIN * n);
  int32_t* counts = ar.alloc<int32_t>(SORT_NBIN);
  HIP_OK(hipMemsetAsync(counts, 0, sizeof(int32_t) * SORT_NBIN, s));
  k_sort_classify<<<nblocks(n, 1024), 1024, 0, s>>>(rp, n, lists, counts);
  // grids sized for the worst case, capped (the kernels walk grid-stride)
  auto grid = [&](int64_t per) { return (unsigned)std::min<int64_t>(nblocks(n, per), 4096); };
  k_sort_group<4><<<grid(64), 256, 0, s>>>(rp, lists + 0 * n, counts + 0, key, src);
  k_sort_group<8><<<grid(32), 256, 0, s>>>(rp, lists + 1 * n, counts + 1, key, src);
  k_sort_group<16><<<grid(16), 256, 0, s>>>(rp, lists + 2 * n, counts + 2, key, src);
  k_sort_group<32><<<grid(8), 256, 0, s>>>(rp, lists + 3 * n, counts + 3, key, src);
  k_sort_group<64><<<grid(4), 256, 0, s>>>(rp, lists + 4 * n, counts + 4, key, src);
  allow_lds((const void*)k_sort_block<SORT_PMAX>);
  const unsigned gb = (unsigned)std::min<int64_t>(n, 2048);
  k_sort_block<512><<<gb, 256, 2 * 512 * sizeof(int32_t), s>>>(rp, lists + 5 * n, counts + 5,
                                                                key, src);
  k_sort_block<2048><<<gb, 256, 2 * 2048 * sizeof(int32_t), s>>>(rp, lists + 6 * n, counts + 6,
                                                                  key, src);
  k_sort_block<SORT_PMAX><<<std::min(gb, 512u), 256, 2 * SORT_PMAX * sizeof(int32_t), s>>>(
      rp, lists + 7 * n, counts + 7, key, src);
  k_sort_global<<<std::min(gb, 64u), 256, 0, s>>>(rp, lists + 8 * n, counts + 8, key, src);
  HIP_OK(hipGetLastError());
}

// Counts and fill of the transpose with one global atomic per distinct
// column and block: a block takes R consecutive rows (about a thousand
// entries), groups their entries by column in an LDS hash table, adds each
// column's count to the global counter (count mode) or reserves that many
// positions on the column's cursor (fill mode) in one atomic, and hands the
// reserved positions out within the block.  The order inside a column is
// arbitrary either way (sort_rows restores it).  A block whose columns do
// not fit the table takes one global atomic per entry instead.
// 32-bit counts and cursors of the transpose (positions below 2^31), one
// global atomic per entry: for matrices whose columns hold few entries
__global__ void k_count_cols32(const int32_t* col, int64_t nnz, uint32_t* cnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[col[e]], 1u);
}

template <int G>
__global__ __launch_bounds__(256) void k_transpose_fill_g(const int64_t* rp, const int32_t* col,
                                                         int64_t n, uint32_t* cursor,
                                                         int32_t* colT, int32_t* src) {
  const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (i >= n) return;
  for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += G) {
    const uint32_t p = atomicAdd(&cursor[col[e]], 1u);
    colT[p] = (int32_t)i;
    src[p] = (int32_t)e;
  }
}

constexpr int TR_HT = 2048;

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ int row_in_block(const int64_t* srp, int nr, int64_t e) {
  int lo = 0, hi = nr - 1;   // the last row r with srp[r] <= e
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (srp[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_transpose_agg(const int64_t* rp, const int32_t* col,
                                                      int64_t n, int R, uint32_t* cc,
                                                      int32_t* colT, int32_t* src) {
  __shared__ int32_t hkey[TR_HT];
  __shared__ uint32_t hcnt[TR_HT];
  __shared__ uint32_t hpos[TR_HT];
  __shared__ int64_t srp[257];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  if (r0 >= n) return;   // (uniform over the block)
  const int nr = (int)(r0 + R < n ? R : n - r0);
  for (int t = tid; t < TR_HT; t += 256) {
    hkey[t] = -1;
    hcnt[t] = 0u;
  }
  for (int t = tid; t <= nr; t += 256) srp[t] = rp[r0 + t];
  if (tid == 0) bad = 0;
  __syncthreads();
  const int64_t e0 = srp[0], e1 = srp[nr];
  for (int64_t e = e0 + tid; e < e1; e += 256) {
    const int32_t c = col[e];
    uint32_t h = hash32((uint32_t)c) & (TR_HT - 1);
    int probes = 0;
    while (true) {
      const int32_t old = atomicCAS(&hkey[h], -1, c);
      if (old == -1 || old == c) {
        atomicAdd(&hcnt[h], 1u);
        break;
      }
      h = (h + 1) & (TR_HT - 1);
      if (++probes >= TR_HT / 4) {
        bad = 1;
        break;
      }
    }
  }
  __syncthreads();
  if (bad) {
    for (int64_t e = e0 + tid; e < e1; e += 256) {
      const int32_t c = col[e];
      const uint32_t p = atomicAdd(&cc[c], 1u);
      if (FILL) {
        colT[p] = (int32_t)(r0 + row_in_block(srp, nr, e));
        src[p] = (int32_t)e;
      }
    }
    return;
  }
  for (int t = tid; t < TR_HT; t += 256) {
    const int32_t c = hkey[t];
    if (c >= 0) {
      const uint32_t k = hcnt[t];
      if (FILL) hpos[t] = atomicAdd(&cc[c], k);
      else atomicAdd(&cc[c], k);
      hcnt[t] = 0u;   // (the fill's counter within the reserved run)
    }
  }
  if (!FILL) return;
  __syncthreads();
  for (int64_t e = e0 + tid; e < e1; e += 256) {
    const int32_t c = col[e];
    uint32_t h = hash32((uint32_t)c) & (TR_HT - 1);
    while (hkey[h] != c) h = (h + 1) & (TR_HT - 1);
    const uint32_t p = hpos[h] + atomicAdd(&hcnt[h], 1u);
    colT[p] = (int32_t)(r0 + row_in_block(srp, nr, e));
    src[p] = (int32_t)e;
  }
}

void transpose_pattern(const CsrView& A, Csr& At, int32_t*& src, hipStream_t s, Arena& ar) {
  At.nrows = A.ncols;
  At.ncols = A.nrows;
  At.nnz = A.nnz;
  if (A.nnz >= INT32_MAX) throw Error(EMIN_ERR_CAPACITY, "transpose: nnz >= 2^31");
  At.rowptr = ar.alloc<int64_t>(At.nrows + 1);
  // (32-bit counts and positions)
  uint32_t* cnt = ar.alloc<uint32_t>(At.nrows > 0 ? At.nrows : 1);
  HIP_OK(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * At.nrows, s));
  HIP_OK(hipMemsetAsync(At.rowptr, 0, sizeof(int64_t), s));
  // block aggregation where a column collects many entries (the transposes
  // of the prolongators: hundreds per coarse point); one atomic per entry
  // where columns hold few (measured: the aggregation is 2x slower there)
  const bool agg = A.ncols > 0 && (double)A.nnz / (double)A.ncols >= 32.0;
  // rows per block: about a thousand entries
  const double avg = A.nrows ? (double)A.nnz / (double)A.nrows : 1.0;
  const int R = (int)std::max(1.0, std::min(256.0, 1024.0 / std::max(avg, 1.0)));
  const unsigned tb = nblocks(A.nrows, R);
  if (A.nnz) {
    if (agg)
      k_transpose_agg<false><<<tb, 256, 0, s>>>(A.rowptr, A.col, A.nrows, R, cnt, nullptr, nullptr);
    else
      k_count_cols32<<<nblocks(A.nnz, 256), 256, 0, s>>>(A.col, A.nnz, cnt);
  }
  if (At.nrows) k_widen_u32<<<nblocks(At.nrows, 256), 256, 0, s>>>(cnt, At.nrows, At.rowptr + 1);
  scan_inclusive(At.rowptr + 1, At.nrows, s, ar);
  At.col = ar.alloc<int32_t>(A.nnz);
  src = ar.alloc<int32_t>(A.nnz);
  uint32_t* cursor = cnt;   // the counts, overwritten with each row's first position
  if (At.nrows) k_narrow_i64<<<nblocks(At.nrows, 256), 256, 0, s>>>(At.rowptr, At.nrows, cursor);
  if (A.nnz) {
    if (agg)
      k_transpose_agg<true><<<tb, 256, 0, s>>>(A.rowptr, A.col, A.nrows, R, cursor, At.col, src);
    else
      ROWS_DISPATCH(lanes_for(A), k_transpose_fill_g, A.nrows, s, A.rowptr, A.col, A.nrows,
                    cursor, At.col, src);
  }
  sort_rows(At.rowptr, At.nrows, At.col, src, s, ar);
}

__global__ void k_gather(const double* in, const int32_t* src, double* out, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = in[src[p]];
}

void gather_values(const double* in, const int32_t* src, double* out, int64_t n, hipStream_t s) {
  if (n) k_gather<<<nblocks(n, 256), 256, 0, s>>>(in, src, out, n);
}

// ---------------------------------------------------------------------------
// SpGEMM, symbolic: G lanes per output row collect the distinct columns in an
// LDS open-addressing table, then write them in ascending order (rank sort).
// ---------------------------------------------------------------------------

// Symbolic pass: a group of G lanes per output row inserts the columns
// reached through A's row into an LDS open-addressing table.  Count mode
// writes the row length; rows whose table would be more than half full are
// appended to ovf (processed again with a larger table).  Fill mode compacts
// the keys and writes them in ascending order (rank of each distinct key).
template <int G, int BS>
__global__ __launch_bounds__(BS) void k_spgemm_sym(const int32_t* rows, int64_t nrows,
                                                   const int64_t* arp, const int32_t* acol,
                                                   const int64_t* brp, const int32_t* bcol,
                                                   int hcap, int64_t* out_cnt, const int64_t* crp,
                                                   int32_t* ccol, int32_t* ovf, int* novf,
                                                   int* derr) {
  extern __shared__ int32_t lds_keys[];
  constexpr int NG = BS / G;
  __shared__ int32_t cnt[NG], cnt2[NG], ovf_g[NG];
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  int32_t* keys = lds_keys + (size_t)g * (hcap + hcap / 2);
  int32_t* dense = keys + hcap;
  const int64_t r = (int64_t)blockIdx.x * NG + g;
  const int64_t row = r < nrows ? (rows ? (int64_t)rows[r] : r) : -1;
  for (int t = lane; t < hcap; t += G) keys[t] = -1;
  if (lane == 0) { cnt[g] = 0; cnt2[g] = 0; ovf_g[g] = 0; }
  __syncthreads();
  const uint32_t mask = (uint32_t)hcap - 1u;
  bool overflow = false;
  if (row >= 0) {
    for (int64_t e = arp[row] + lane; e < arp[row + 1] && !overflow; e += G) {
      const int32_t k = acol[e];
      for (int64_t f = brp[k]; f < brp[k + 1]; f++) {
        const int32_t j = bcol[f];
        uint32_t h = hash32((uint32_t)j) & mask;
        int probes = 0;
        while (true) {
          const int32_t old = atomicCAS(&keys[h], -1, j);
          if (old == -1) {
            if (atomicAdd(&cnt[g], 1) >= hcap / 2) overflow = true;
            break;
          }
          if (old == j) break;
          h = (h + 1u) & mask;
          if (++probes >= hcap) { overflow = true; break; }
        }
        if (overflow) break;
      }
    }
  }
  if (overflow) atomicOr(&ovf_g[g], 1);
  __syncthreads();
  if (row < 0) return;
  const bool over = ovf_g[g] != 0 || cnt[g] > hcap / 2;
  if (ccol == nullptr) {
    if (lane == 0) {
      if (over) {
        if (ovf) ovf[atomicAdd(novf, 1)] = (int32_t)row;
        else atomicOr(derr, DERR_CAPACITY);
      } else {
        out_cnt[row + 1] = cnt[g];
      }
    }
    return;
  }
  if (over) {
    // the caller redoes overflowed rows with a larger table; without that
    // second pass (ovf == nullptr only there) this is an error
    if (lane == 0 && ovf == nullptr && rows != nullptr) atomicOr(derr, DERR_CAPACITY);
    return;
  }
  for (int t = lane; t < hcap; t += G) {
    const int32_t key = keys[t];
    if (key >= 0) dense[atomicAdd(&cnt2[g], 1)] = key;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int u = cnt[g];
  const int64_t base = crp[row];
  for (int t = lane; t < u; t += G) {
    const int32_t key = dense[t];
    int rank = 0;
    for (int v = 0; v < u; v++) rank += dense[v] < key;
    ccol[base + rank] = key;
  }
}

// Numeric product, G lanes per output row (a group never spans two waves).
// The row's accumulators sit in LDS together with an index of its sorted
// columns that maps a column j to its slot:
//   flat window (span of nw words fits): word w holds the row's column bits
//     and the slot of its first column, slot = first + popc(bits below j);
//   two-level (nw1 = nw/32 super-words plus one pair per non-empty word
//     fit): super-word s holds the bits of its non-empty words and the rank
//     of the first one, which picks the word's pair as above;
//   otherwise a binary search over the sorted columns.
// The slots of a batch of consecutive A entries are found first (independent
// lookups), then their products are added (acc_add).  The entries of one B
// row land in distinct slots, and a wave's LDS operations complete in issue
// order, so every c_ij still receives its products in ascending order of A's
// row, each product and each sum rounded separately.
// orders a group's LDS writes before its later reads: the group lies inside
// one wave, whose LDS operations complete in issue order, so a wave-scope
// fence (a compiler barrier, no wait on outstanding global loads) suffices
template <int G>
__device__ __forceinline__ void group_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// split rows of a numeric product (see SpgemmPlan)
template <class TV>
struct SplitArgsT {
  const int32_t* trow = nullptr;
  const int32_t* tchunk = nullptr;
  const int64_t* poff = nullptr;
  TV* part = nullptr;
  int64_t ntasks = 0;
};

// acc[slot] += v, in the wave's issue order.  FP64: an LDS atomic add (no
// return, so consecutive adds do not wait for each other).  FP32: a plain
// read-add-write (measured faster than the LDS float atomic here); a wave's
// LDS operations complete in order, and acc_order(), called by every lane
// after each entry's adds, keeps the compiler from moving the next entry's
// reads above these writes.
template <class TV>
__device__ __forceinline__ void acc_add(TV* acc, int slot, TV v) {
  if constexpr (sizeof(TV) == 8) atomicAdd(&acc[slot], v);
  else acc[slot] = acc[slot] + v;
}

template <class TV>
__device__ __forceinline__ void acc_order() {
  if constexpr (sizeof(TV) == 4) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int G, class TV, class TO>
__global__ __launch_bounds__(256) void k_spgemm_num(const int64_t* arp, const int32_t* acol,
                                                   const TV* aval, const int64_t* brp,
                                                   const int32_t* bcol, const TV* bval,
                                                   const int64_t* crp, const int32_t* ccol,
                                                   TO* cval, int64_t n, int cap, int iw,
                                                   SplitArgsT<TV> sp) {
  extern __shared__ uint32_t lds_words[];
  constexpr int NG = 256 / G;
  constexpr int UF = G < 16 ? G : 16;   // A entries per batch when B rows fit the group
  constexpr int US = 4;                 // ... when some B row is longer than the group
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t* idx = lds_words + (size_t)g * iw;   // iw even: pairs stay 8-byte aligned
  TV* acc = reinterpret_cast<TV*>(lds_words + (size_t)NG * iw) + (size_t)g * cap;
  // (measured: the dispatch order beats the XCD-contiguous one here, although
  // the latter raises the L2 hit rate)
  // row mode: one output row per group (split rows are left to the chunk
  // items); chunk mode (sp.trow set): one chunk of a split row per group,
  // its sums written to sp.part
  int64_t row, ea, eb;
  TV* pout = nullptr;
  if (sp.trow) {
    const int64_t w = (int64_t)blockIdx.x * NG + g;
    if (w >= sp.ntasks) return;
    row = sp.trow[w];
    const int64_t ch = sp.tchunk[w];
    ea = arp[row] + ch * SPGEMM_SPLIT;
    eb = ea + SPGEMM_SPLIT < arp[row + 1] ? ea + SPGEMM_SPLIT : arp[row + 1];
    pout = sp.part + sp.poff[row] + ch * (crp[row + 1] - crp[row]);
  } else {
    row = (int64_t)blockIdx.x * NG + g;
    if (row >= n) return;
    if (sp.poff && sp.poff[row] >= 0) return;
    ea = arp[row];
    eb = arp[row + 1];
  }
  const int64_t c0 = crp[row];
  const int nc = (int)(crp[row + 1] - c0);
  if (nc > cap || nc == 0) return;  // long rows: k_spgemm_num_long
  const int32_t jlo = ccol[c0];
  const int64_t span = (int64_t)ccol[c0 + nc - 1] - jlo;
  const int64_t nw = (span >> 5) + 1, nw1 = (nw + 31) >> 5;
  // 1: flat window, 2: two-level, 0: binary search (uniform over the group)
  const int mode = 2 * nw <= iw ? 1 : (2 * (nw1 + nc) <= iw ? 2 : 0);
  uint32_t* cw = idx + 2 * nw1;   // two-level: pairs of the non-empty words
  for (int t = lane; t < nc; t += G) acc[t] = TV(0);
  if (mode == 1) {
    for (int t = lane; t < nw; t += G) idx[2 * t] = 0u;
  } else if (mode == 2) {
    for (int t = lane; t < nw1; t += G) idx[2 * t] = 0u;
    for (int t = lane; t < nc; t += G) cw[2 * t] = 0u;
  } else {
    for (int t = lane; t < nc; t += G) idx[t] = (uint32_t)ccol[c0 + t];
  }
  group_sync_lds<G>();
  if (mode == 1) {
    for (int t = lane; t < nc; t += G) {
      const int r = ccol[c0 + t] - jlo;
      const int w = r >> 5;
      atomicOr(&idx[2 * w], 1u << (r & 31));
      if (t == 0 || ((ccol[c0 + t - 1] - jlo) >> 5) != w) idx[2 * w + 1] = (uint32_t)t;
    }
    group_sync_lds<G>();
  } else if (mode == 2) {
    for (int t = lane; t < nc; t += G) {
      const int w = (ccol[c0 + t] - jlo) >> 5;
      atomicOr(&idx[2 * (w >> 5)], 1u << (w & 31));
    }
    group_sync_lds<G>();
    // rank of each super-word's first non-empty word (exclusive scan)
    int run = 0;
    for (int s0 = 0; s0 < nw1; s0 += G) {
      const int sw = s0 + lane;
      const int c = sw < nw1 ? __popc(idx[2 * sw]) : 0;
      int incl = c;
#pragma unroll
      for (int m = 1; m < G; m <<= 1) {
        const int o = __shfl_up(incl, m, G);
        if (lane >= m) incl += o;
      }
      if (sw < nw1) idx[2 * sw + 1] = (uint32_t)(run + incl - c);
      run += __shfl(incl, G - 1, G);
    }
    group_sync_lds<G>();
    for (int t = lane; t < nc; t += G) {
      const int r = ccol[c0 + t] - jlo;
      const int w = r >> 5, sw = w >> 5;
      const int d = (int)idx[2 * sw + 1] + __popc(idx[2 * sw] & ((1u << (w & 31)) - 1u));
      atomicOr(&cw[2 * d], 1u << (r & 31));
      if (t == 0 || ((ccol[c0 + t - 1] - jlo) >> 5) != w) cw[2 * d + 1] = (uint32_t)t;
    }
    group_sync_lds<G>();
  }
  auto slot_of = [&](int32_t j) -> int {
    const int r = j - jlo;
    if (mode == 1) {
      const uint2 e = *reinterpret_cast<const uint2*>(idx + 2 * (r >> 5));
      return (int)e.y + __popc(e.x & ((1u << (r & 31)) - 1u));
    }
    if (mode == 2) {
      const int w = r >> 5;
      const uint2 e1 = *reinterpret_cast<const uint2*>(idx + 2 * (w >> 5));
      const int d = (int)e1.y + __popc(e1.x & ((1u << (w & 31)) - 1u));
      const uint2 e2 = *reinterpret_cast<const uint2*>(cw + 2 * d);
      return (int)e2.y + __popc(e2.x & ((1u << (r & 31)) - 1u));
    }
    int lo = 0, hi = nc;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((int32_t)idx[mid] < j) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  // A entries of the next chunk are loaded while the current one is summed
  int32_t kk_n = 0;
  TV av_n = TV(0);
  int64_t kb0_n = 0;
  int kl_n = 0;
  if (ea + lane < eb) {
    kk_n = acol[ea + lane];
    av_n = aval[ea + lane];
    kb0_n = brp[kk_n];
    kl_n = (int)(brp[kk_n + 1] - kb0_n);
  }
  for (int64_t e0 = ea; e0 < eb; e0 += G) {
    const TV av = av_n;
    const int64_t kb0 = kb0_n;
    const int kl = kl_n;
    const int cnt = (int)((eb - e0) < G ? (eb - e0) : G);
    {
      const int64_t e = e0 + G + lane;
      kl_n = 0;
      if (e < eb) {
        kk_n = acol[e];
        av_n = aval[e];
        kb0_n = brp[kk_n];
        kl_n = (int)(brp[kk_n + 1] - kb0_n);
      }
    }
    if (group_ballot<G>(kl > G) == 0ull) {
      // every B row of the chunk fits the group: one entry per lane
      for (int q0 = 0; q0 < cnt; q0 += UF) {
        int32_t jj[UF];
        TV pr[UF];
#pragma unroll
        for (int u = 0; u < UF; u++) {
          const int q = q0 + u;
          const int64_t b0 = __shfl(kb0, q, G);
          const int bl = q < cnt ? __shfl(kl, q, G) : 0;
          const TV am = __shfl(av, q, G);
          jj[u] = lane < bl ? bcol[b0 + lane] : -1;
          pr[u] = am * (lane < bl ? bval[b0 + lane] : TV(0));
        }
        int sl[UF];
#pragma unroll
        for (int u = 0; u < UF; u++) sl[u] = jj[u] >= 0 ? slot_of(jj[u]) : -1;
#pragma unroll
        for (int u = 0; u < UF; u++) {
          if (sl[u] >= 0) acc_add(acc, sl[u], pr[u]);
          acc_order<TV>();
        }
      }
    } else {
      for (int q0 = 0; q0 < cnt; q0 += US) {
        int32_t jj[US];
        TV bv[US], am[US];
        int64_t b0[US];
        int bl[US], sl[US];
#pragma unroll
        for (int u = 0; u < US; u++) {
          const int q = q0 + u;
          b0[u] = __shfl(kb0, q, G);
          bl[u] = q < cnt ? __shfl(kl, q, G) : 0;
          am[u] = __shfl(av, q, G);
          jj[u] = lane < bl[u] ? bcol[b0[u] + lane] : -1;
          bv[u] = lane < bl[u] ? bval[b0[u] + lane] : TV(0);
        }
#pragma unroll
        for (int u = 0; u < US; u++) sl[u] = jj[u] >= 0 ? slot_of(jj[u]) : 0;
#pragma unroll
        for (int u = 0; u < US; u++) {
          if (jj[u] >= 0) acc_add(acc, sl[u], am[u] * bv[u]);
          // the rest of a B row longer than the group, before the next entry
          for (int off = G; off < bl[u]; off += G) {
            if (off + lane < bl[u]) {
              const int32_t j = bcol[b0[u] + off + lane];
              const TV b = bval[b0[u] + off + lane];
              acc_add(acc, slot_of(j), am[u] * b);
            }
          }
          acc_order<TV>();
        }
      }
    }
  }
  group_sync_lds<G>();
  if (pout) {
    for (int t = lane; t < nc; t += G) pout[t] = acc[t];
  } else {
    for (int t = lane; t < nc; t += G) cval[c0 + t] = (TO)acc[t];
  }
}

// split rows: c_it = the chunk sums of slot t added in chunk order (one
// group of 64 lanes per split row, found as its chunk-0 work item)
template <class TV, class TO>
__global__ __launch_bounds__(256) void k_spgemm_combine(const int64_t* arp, const int64_t* crp,
                                                       SplitArgsT<TV> sp, TO* cval) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= sp.ntasks || sp.tchunk[w] != 0) return;
  const int64_t row = sp.trow[w];
  const int64_t c0 = crp[row], nc = crp[row + 1] - c0;
  const int64_t nch = (arp[row + 1] - arp[row] + SPGEMM_SPLIT - 1) / SPGEMM_SPLIT;
  const TV* p = sp.part + sp.poff[row];
  for (int64_t t = lane; t < nc; t += 64) {
    TV v = p[t];
    for (int64_t c = 1; c < nch; c++) v = v + p[c * nc + t];
    cval[c0 + t] = (TO)v;
  }
}

// fallback for rows longer than the LDS capacity: one lane per row, the
// accumulators live in the output array itself (same summation order)
template <class TV, class TO>
__global__ void k_spgemm_num_long(const int64_t* arp, const int32_t* acol, const TV* aval,
                                  const int64_t* brp, const int32_t* bcol, const TV* bval,
                                  const int64_t* crp, const int32_t* ccol, TO* cval,
                                  int64_t n, int cap) {
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const int64_t c0 = crp[row];
  const int nc = (int)(crp[row + 1] - c0);
  if (nc <= cap) return;
  TV accv = TV(0);
  (void)accv;
  for (int t = 0; t < nc; t++) cval[c0 + t] = TO(0);
  for (int64_t e = arp[row]; e < arp[row + 1]; e++) {
    const int32_t k = acol[e];
    const TV a = aval[e];
    for (int64_t f = brp[k]; f < brp[k + 1]; f++) {
      const int32_t j = bcol[f];
      int lo = 0, hi = nc;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (ccol[c0 + mid] < j) lo = mid + 1; else hi = mid;
      }
      const TV prod = a * bval[f];
      cval[c0 + lo] = (TO)((TV)cval[c0 + lo] + prod);
    }
  }
}

// maximum over a 256-thread block, then one atomic per block
__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long* mx) {
  __shared__ unsigned long long part[4];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long o = __shfl_xor(v, m, 64);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; w++) v = part[w] > v ? part[w] : v;
    atomicMax(mx, v);
  }
}

__global__ __launch_bounds__(256) void k_row_len_max(const int64_t* rp, int64_t n,
                                                    unsigned long long* mx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  block_max_to(i < n ? (unsigned long long)(rp[i + 1] - rp[i]) : 0ull, mx);
}

// longest row and widest window of a symbolic product: block maxima, one
// atomic pair per block
// chunks of a row summed apart (0: the row is not split)
__device__ __forceinline__ int64_t split_chunks(int64_t lena, int64_t nc) {
  return (lena > SPGEMM_SPLIT && nc > 0 && nc <= SPGEMM_SPLIT_NC)
             ? (lena + SPGEMM_SPLIT - 1) / SPGEMM_SPLIT : 0;
}

// mx[0] longest row, mx[1] widest window, mx[4] longest row of A (block
// maxima, one atomic each per block); mx[2] split work items and mx[3]
// chunk-sum values (block sums; arp null: no split)
__global__ __launch_bounds__(256) void k_sym_maxima(const int64_t* rp, const int32_t* rwords,
                                                   const int64_t* arp, const int64_t* aall,
                                                   int64_t n, unsigned long long* mx) {
  __shared__ unsigned long long part[5][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nc = i < n ? rp[i + 1] - rp[i] : 0;
  unsigned long long la = i < n ? (unsigned long long)(aall[i + 1] - aall[i]) : 0ull;
  unsigned long long a = (unsigned long long)nc;
  unsigned long long b = i < n ? (unsigned long long)rwords[i] : 0ull;
  const int64_t ch = (i < n && arp) ? split_chunks(arp[i + 1] - arp[i], nc) : 0;
  unsigned long long c = (unsigned long long)ch, d = (unsigned long long)(ch * nc);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const unsigned long long oa = __shfl_xor(a, m, 64), ob = __shfl_xor(b, m, 64);
    a = oa > a ? oa : a;
    b = ob > b ? ob : b;
    c += __shfl_xor(c, m, 64);
    d += __shfl_xor(d, m, 64);
    const unsigned long long ol = __shfl_xor(la, m, 64);
    la = ol > la ? ol : la;
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = a;
    part[1][threadIdx.x >> 6] = b;
    part[2][threadIdx.x >> 6] = c;
    part[3][threadIdx.x >> 6] = d;
    part[4][threadIdx.x >> 6] = la;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long v = part[threadIdx.x][0];
    for (int w = 1; w < 4; w++) v = part[threadIdx.x][w] > v ? part[threadIdx.x][w] : v;
    atomicMax(&mx[threadIdx.x], v);
  } else if (threadIdx.x < 4) {
    const unsigned long long v = part[threadIdx.x][0] + part[threadIdx.x][1] +
                                 part[threadIdx.x][2] + part[threadIdx.x][3];
    if (v) atomicAdd(&mx[threadIdx.x], v);
  } else if (threadIdx.x == 4) {
    unsigned long long v = part[4][0];
    for (int w = 1; w < 4; w++) v = part[4][w] > v ? part[4][w] : v;
    atomicMax(&mx[4], v);
  }
}

// per row: its chunk count and chunk-sum values (scanned afterwards)
__global__ void k_split_counts(const int64_t* rp, const int64_t* arp, int64_t n, int64_t* ch,
                               int64_t* vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t nc = rp[i + 1] - rp[i];
  const int64_t c = split_chunks(arp[i + 1] - arp[i], nc);
  ch[i] = c;
  vals[i] = c * nc;
}

__global__ void k_split_fill(const int64_t* rp, const int64_t* ch_incl, const int64_t* val_incl,
                             int64_t n, int32_t* trow, int32_t* tchunk, int64_t* poff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c1 = ch_incl[i], c0 = i ? ch_incl[i - 1] : 0;
  if (c1 == c0) {
    poff[i] = -1;
    return;
  }
  poff[i] = val_incl[i] - (c1 - c0) * (rp[i + 1] - rp[i]);
  for (int64_t c = c0; c < c1; c++) {
    trow[c] = (int32_t)i;
    tchunk[c] = (int32_t)(c - c0);
  }
}

// output size, count-pass overflow flag, longest row, widest window, split
// work items and chunk-sum values
__global__ void k_sym_summary(const int64_t* rp, int64_t n, const int* lerr,
                              const unsigned long long* mx, int64_t* out) {
  if (threadIdx.x == 0) {
    out[0] = rp[n];
    out[1] = lerr[0];
    out[2] = (int64_t)mx[0];
    out[3] = (int64_t)mx[1];
    out[4] = (int64_t)mx[2];
    out[5] = (int64_t)mx[3];
    out[6] = (int64_t)mx[4];
  }
}

// a fill-pass overflow is reported with the handle's other deferred errors
__global__ void k_defer_err(const int* lerr, int* derr) {
  if (threadIdx.x == 0 && lerr[0]) atomicOr(derr, DERR_CAPACITY);
}

void max_row_len_dev(const int64_t* rp, int64_t n, unsigned long long* out, hipStream_t s) {
  HIP_OK(hipMemsetAsync(out, 0, sizeof(unsigned long long), s));
  if (n > 0) k_row_len_max<<<nblocks(n, 256), 256, 0, s>>>(rp, n, out);
}

int64_t max_row_len(const int64_t* rp, int64_t n, hipStream_t s, Arena& ar) {
  if (n <= 0) return 0;
  unsigned long long* mx = ar.alloc<unsigned long long>(1);
  max_row_len_dev(rp, n, mx, s);
  return (int64_t)d2h(mx, s);
}

__global__ __launch_bounds__(256) void k_max_i32(const int32_t* a, int64_t n,
                                                unsigned long long* mx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  block_max_to(i < n ? (unsigned long long)a[i] : 0ull, mx);
}

int64_t max_row_len_i32(const int32_t* a, int64_t n, hipStream_t s, Arena& ar) {
  if (n <= 0) return 0;
  unsigned long long* mx = ar.alloc<unsigned long long>(1);
  HIP_OK(hipMemsetAsync(mx, 0, sizeof(unsigned long long), s));
  k_max_i32<<<nblocks(n, 256), 256, 0, s>>>(a, n, mx);
  return (int64_t)d2h(mx, s);
}

static int pick_g(double avg) {
  int g = 4;
  while (g < 64 && g < avg) g <<= 1;
  return g;
}

template <int G, int BS>
static void launch_sym(const int32_t* rows, int64_t nrows, const CsrView& A, const CsrView& B,
                       int hcap, int64_t* cnt, const int64_t* crp, int32_t* ccol, int32_t* ovf,
                       int* novf, int* derr, hipStream_t s) {
  constexpr int NG = BS / G;
  const size_t lds = (size_t)NG * (hcap + hcap / 2) * sizeof(int32_t);
  allow_lds((const void*)k_spgemm_sym<G, BS>);
  k_spgemm_sym<G, BS><<<nblocks(nrows, NG), BS, lds, s>>>(rows, nrows, A.rowptr, A.col, B.rowptr,
                                                          B.col, hcap, cnt, crp, ccol, ovf, novf,
                                                          derr);
}

static void sym_dispatch(int g, int64_t nrows, const CsrView& A, const CsrView& B, int hcap,
                         int64_t* cnt, const int64_t* crp, int32_t* ccol, int32_t* ovf, int* novf,
                         int* derr, hipStream_t s) {
  switch (g) {
    case 4: launch_sym<4, 256>(nullptr, nrows, A, B, hcap, cnt, crp, ccol, ovf, novf, derr, s); break;
    case 8: launch_sym<8, 256>(nullptr, nrows, A, B, hcap, cnt, crp, ccol, ovf, novf, derr, s); break;
    case 16: launch_sym<16, 256>(nullptr, nrows, A, B, hcap, cnt, crp, ccol, ovf, novf, derr, s); break;
    case 32: launch_sym<32, 256>(nullptr, nrows, A, B, hcap, cnt, crp, ccol, ovf, novf, derr, s); break;
    default: launch_sym<64, 256>(nullptr, nrows, A, B, hcap, cnt, crp, ccol, ovf, novf, derr, s); break;
  }
}

// rows whose table overflowed: one 64-lane group per block, a large table
static void sym_big(const int32_t* rows, int64_t nrows, const CsrView& A, const CsrView& B,
                    int hcap, int64_t* cnt, const int64_t* crp, int32_t* ccol, int* derr,
                    hipStream_t s) {
  if (nrows)
    launch_sym<64, 64>(rows, nrows, A, B, hcap, cnt, crp, ccol, nullptr, nullptr, derr, s);
}

// Symbolic pass over a column window: a row's output columns all lie between
// the smallest first column and the largest last column of the B rows its
// A entries select (B rows are sorted).  When that window is at most
// 32 * wcap columns wide, a visited bitmap over it replaces the hash table:
// one atomic OR per product, no probing, and the set bits read out in order
// give the sorted row directly.  Rows with a wider window are listed in ovf
// (count mode) or skipped (fill mode) and go to the hash kernels.
template <int G>
__global__ __launch_bounds__(256) void k_spgemm_win(int64_t n, const int64_t* arp,
                                                   const int32_t* acol, const int64_t* brp,
                                                   const int32_t* bcol, int wcap,
                                                   int64_t* out_cnt, const int64_t* crp,
                                                   int32_t* ccol, int32_t* ovf, int* novf,
                                                   int32_t* rwords) {
  extern __shared__ uint32_t sbits[];
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t* words = sbits + (size_t)g * wcap;
  const int64_t row = xcd_block(blockIdx.x, gridDim.x) * NG + g;
  if (row >= n) return;   // whole group; the block never synchronises
  const int64_t ea = arp[row], eb = arp[row + 1];
  // window bounds
  int32_t lo = INT32_MAX, hi = -1;
  for (int64_t e = ea + lane; e < eb; e += G) {
    const int32_t k = acol[e];
    const int64_t b0 = brp[k], b1 = brp[k + 1];
    if (b1 > b0) {
      const int32_t f = bcol[b0], l = bcol[b1 - 1];
      lo = f < lo ? f : lo;
      hi = l > hi ? l : hi;
    }
  }
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) {
    const int32_t ol = __shfl_xor(lo, m, G), oh = __shfl_xor(hi, m, G);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  if (hi < 0) {   // empty output row
    if (out_cnt && lane == 0) {
      out_cnt[row + 1] = 0;
      rwords[row] = 0;
    }
    return;
  }
  const int64_t width = (int64_t)hi - lo + 1;
  // lo and hi are columns of the output row, so nw is also the word count of
  // the numeric pass's window over that row
  const int nw = (int)((width + 31) >> 5);
  if (out_cnt && lane == 0) rwords[row] = nw;
  if (nw > wcap) {
    if (out_cnt && lane == 0) ovf[atomicAdd(novf, 1)] = (int32_t)row;
    return;
  }
  for (int t = lane; t < nw; t += G) words[t] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int64_t e = ea + lane; e < eb; e += G) {
    const int32_t k = acol[e];
    const int64_t b0 = brp[k], b1 = brp[k + 1];
    for (int64_t f = b0; f < b1; f += 4) {
      int32_t j[4];
#pragma unroll
      for (int q = 0; q < 4; q++) j[q] = f + q < b1 ? bcol[f + q] - lo : -1;
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (j[q] >= 0) atomicOr(&words[j[q] >> 5], 1u << (j[q] & 31));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // lane l owns words [l*wpl, (l+1)*wpl)
  const int wpl = (nw + G - 1) / G;
  const int w0 = lane * wpl, w1 = (w0 + wpl) < nw ? (w0 + wpl) : nw;
  int c = 0;
  for (int t = w0; t < w1; t++) c += __popc(words[t]);
  int incl = c;   // inclusive scan over the group
#pragma unroll
  for (int m = 1; m < G; m <<= 1) {
    const int o = __shfl_up(incl, m, G);
    if (lane >= m) incl += o;
  }
  const int total = __shfl(incl, G - 1, G);
  if (out_cnt) {
    if (lane == 0) out_cnt[row + 1] = total;
    return;
  }
  int32_t* out = ccol + crp[row] + (incl - c);
  for (int t = w0; t < w1; t++) {
    uint32_t m = words[t];
    while (m) {
      const int b = __builtin_ctz(m);
      m &= m - 1u;
      *out++ = lo + 32 * t + b;
    }
  }
}

template <int G>
static void launch_win(int64_t n, const CsrView& A, const CsrView& B, int wcap, int64_t* cnt,
                       const int64_t* crp, int32_t* ccol, int32_t* ovf, int* novf,
                       int32_t* rwords, hipStream_t s) {
  constexpr int NG = 256 / G;
  const size_t lds = (size_t)NG * wcap * sizeof(uint32_t);
  allow_lds((const void*)k_spgemm_win<G>);
  k_spgemm_win<G><<<nblocks(n, NG), 256, lds, s>>>(n, A.rowptr, A.col, B.rowptr, B.col, wcap,
                                                   cnt, crp, ccol, ovf, novf, rwords);
}

static void win_dispatch(int g, int64_t n, const CsrView& A, const CsrView& B, int wcap,
                         int64_t* cnt, const int64_t* crp, int32_t* ccol, int32_t* ovf, int* novf,
                         int32_t* rwords, hipStream_t s) {
  switch (g) {
    case 4: launch_win<4>(n, A, B, wcap, cnt, crp, ccol, ovf, novf, rwords, s); break;
    case 8: launch_win<8>(n, A, B, wcap, cnt, crp, ccol, ovf, novf, rwords, s); break;
    case 16: launch_win<16>(n, A, B, wcap, cnt, crp, ccol, ovf, novf, rwords, s); break;
    case 32: launch_win<32>(n, A, B, wcap, cnt, crp, ccol, ovf, novf, rwords, s); break;
    default: launch_win<64>(n, A, B, wcap, cnt, crp, ccol, ovf, novf, rwords, s); break;
  }
}

// The same window method with the bitmaps kept: k_spgemm_bounds finds each
// output row's window once (rows wider than wcap words are listed in ovf for
// the hash kernels and keep no words), k_spgemm_bits builds the bitmap in
// LDS, counts it and stores its words at the row's offset in a scratch
// buffer, and k_spgemm_expand turns the stored words into the sorted column
// list once the row pointers are known.  The products of A and B are formed
// once instead of once per pass.
template <int G>
__global__ __launch_bounds__(256) void k_spgemm_bounds(int64_t n, const int64_t* arp,
                                                      const int32_t* acol, const int64_t* brp,
                                                      const int32_t* bcol, int wcap,
                                                      int32_t* rlo, int32_t* rwords,
                                                      int64_t* wcnt, int32_t* ovf, int* novf) {
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t row = xcd_block(blockIdx.x, gridDim.x) * NG + g;
  if (row < n) {
    const int64_t ea = arp[row], eb = arp[row + 1];
    int32_t lo = INT32_MAX, hi = -1;
    // four A entries per lane at a time, their loads issued together
    for (int64_t e0 = ea + lane; e0 < eb; e0 += 4 * G) {
      int32_t k[4];
      int64_t b0[4], b1[4];
#pragma unroll
      for (int q = 0; q < 4; q++) k[q] = e0 + q * G < eb ? acol[e0 + q * G] : -1;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        b0[q] = k[q] >= 0 ? brp[k[q]] : 0;
        b1[q] = k[q] >= 0 ? brp[k[q] + 1] : 0;
      }
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (b1[q] > b0[q]) {
          const int32_t f = bcol[b0[q]], l = bcol[b1[q] - 1];
          lo = f < lo ? f : lo;
          hi = l > hi ? l : hi;
        }
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
      const int32_t ol = __shfl_xor(lo, m, G), oh = __shfl_xor(hi, m, G);
      lo = ol < lo ? ol : lo;
      hi = oh > hi ? oh : hi;
    }
    if (lane == 0) {
      if (hi < 0) {
        rlo[row] = 0;
        rwords[row] = 0;
        wcnt[row] = 0;
      } else {
        const int nw = (int)((((int64_t)hi - lo + 1) + 31) >> 5);
        rlo[row] = lo;
        rwords[row] = nw;
        if (nw > wcap) {
          ovf[atomicAdd(novf, 1)] = (int32_t)row;
          wcnt[row] = 0;
        } else {
          wcnt[row] = nw;
        }
      }
    }
  }
}

// the widest stored window (block maxima, one atomic per 1024 rows)
__global__ __launch_bounds__(256) void k_wcnt_max(const int64_t* wcnt, int64_t n,
                                                 unsigned long long* mx) {
  __shared__ unsigned long long part[4];
  int64_t best = 0;
  for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
       i < n && i < (int64_t)(blockIdx.x + 1) * 1024; i += 256)
    best = wcnt[i] > best ? wcnt[i] : best;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int64_t o = __shfl_xor(best, m, 64);
    best = o > best ? o : best;
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = (unsigned long long)best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long v = part[0];
    for (int w = 1; w < 4; w++) v = part[w] > v ? part[w] : v;
    if (v) atomicMax(mx, v);
  }
}

// MODE 0: a lane per A entry walking its B row; 1: flattened B rows; 2: four
// A entries per lane with the first eight entries of their B rows loaded
// together (short B rows, several rows of C per wave)
// nsl > 1 (sliced form, for few long rows): nsl groups per row, each taking
// an equal share of the row's A entries and OR-ing its bitmap into the row's
// stored words (zeroed beforehand); the counts then come from
// k_spgemm_bits_count
template <int G, int MODE>
__global__ __launch_bounds__(256) void k_spgemm_bits(int64_t n, const int64_t* arp,
                                                    const int32_t* acol, const int64_t* brp,
                                                    const int32_t* bcol, int wlds, int wcap,
                                                    const int32_t* rlo, const int32_t* rwords,
                                                    const int64_t* wincl, uint32_t* wbuf,
                                                    int64_t* out_cnt, int nsl = 1) {
  extern __shared__ uint32_t sbits[];
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  uint32_t* words = sbits + (size_t)g * wlds;
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * NG + g;
  const int64_t row = gid / nsl;
  const int sl = (int)(gid - row * nsl);
  if (row >= n) return;   // whole group; the block never synchronises
  const int nw = rwords[row];
  if (nw == 0 || nw > wcap) return;   // empty (count stays 0), or a hash-kernel row
  const int32_t lo = rlo[row];
  for (int t = lane; t < nw; t += G) words[t] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int64_t ea = arp[row], eb = arp[row + 1];
  if (nsl > 1) {
    const int64_t len = eb - ea, a0 = ea;
    ea = a0 + len * sl / nsl;
    eb = a0 + len * (sl + 1) / nsl;
  }
  if (MODE == 2) {
    for (int64_t e0 = ea + lane; e0 < eb; e0 += 4 * G) {
      int32_t k[4];
      int64_t b0[4];
      int len[4];
#pragma unroll
      for (int q = 0; q < 4; q++) k[q] = e0 + q * G < eb ? acol[e0 + q * G] : -1;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        b0[q] = k[q] >= 0 ? brp[k[q]] : 0;
        len[q] = k[q] >= 0 ? (int)(brp[k[q] + 1] - b0[q]) : 0;
      }
      int32_t j[4][8];
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int t = 0; t < 8; t++) j[q][t] = t < len[q] ? bcol[b0[q] + t] - lo : -1;
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int t = 0; t < 8; t++)
          if (j[q][t] >= 0) atomicOr(&words[j[q][t] >> 5], 1u << (j[q][t] & 31));
#pragma unroll
      for (int q = 0; q < 4; q++)
        for (int t = 8; t < len[q]; t++) {
          const int32_t jj = bcol[b0[q] + t] - lo;
          atomicOr(&words[jj >> 5], 1u << (jj & 31));
        }
    }
  } else if (MODE == 0) {
    // lane per A entry, walking its B row
    for (int64_t e = ea + lane; e < eb; e += G) {
      const int32_t k = acol[e];
      const int64_t b0 = brp[k], b1 = brp[k + 1];
      for (int64_t f = b0; f < b1; f += 4) {
        int32_t j[4];
#pragma unroll
        for (int q = 0; q < 4; q++) j[q] = f + q < b1 ? bcol[f + q] - lo : -1;
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (j[q] >= 0) atomicOr(&words[j[q] >> 5], 1u << (j[q] & 31));
      }
    }
  } else {
    // the B rows of G consecutive A entries, flattened: lane t takes entries
    // t, t + G, ... of their concatenation (the owner of entry f is the
    // first lane whose inclusive length sum exceeds f)
    for (int64_t e0 = ea; e0 < eb; e0 += G) {
      const int64_t e = e0 + lane;
      int64_t b0 = 0;
      int len = 0;
      if (e < eb) {
        const int32_t k = acol[e];
        b0 = brp[k];
        len = (int)(brp[k + 1] - b0);
      }
      int incl = len;
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const int o = __shfl_up(incl, d, G);
        if (lane >= d) incl += o;
      }
      const int total = __shfl(incl, G - 1, G);
      const int excl = incl - len;
      for (int f0 = 0; f0 < total; f0 += G) {
        const int f = f0 + lane;
        int pos = 0;
#pragma unroll
        for (int st = G / 2; st >= 1; st >>= 1)
          if (__shfl(incl, pos + st - 1, G) <= f) pos += st;
        const int64_t sb = __shfl(b0, pos, G);
        const int se = __shfl(excl, pos, G);
        if (f < total) {
          const int32_t j = bcol[sb + (f - se)] - lo;
          atomicOr(&words[j >> 5], 1u << (j & 31));
        }
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t* dst = wbuf + (wincl[row] - nw);
  if (nsl > 1) {
    for (int t = lane; t < nw; t += G) {
      const uint32_t wv = words[t];
      if (wv) atomicOr(&dst[t], wv);
    }
    return;
  }
  int c = 0;
  for (int t = lane; t < nw; t += G) {
    const uint32_t wv = words[t];
    c += __popc(wv);
    dst[t] = wv;
  }
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) c += __shfl_xor(c, m, G);
  if (lane == 0) out_cnt[row + 1] = c;
}

// entries of each row of the sliced form: the set bits of its stored words
template <int G>
__global__ __launch_bounds__(256) void k_spgemm_bits_count(int64_t n, int wcap,
                                                          const int32_t* rwords,
                                                          const int64_t* wincl,
                                                          const uint32_t* wbuf,
                                                          int64_t* out_cnt) {
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t row = (int64_t)blockIdx.x * NG + g;
  if (row >= n) return;
  const int nw = rwords[row];
  if (nw == 0 || nw > wcap) return;
  const uint32_t* src = wbuf + (wincl[row] - nw);
  int c = 0;
  for (int t = lane; t < nw; t += G) c += __popc(src[t]);
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) c += __shfl_xor(c, m, G);
  if (lane == 0) out_cnt[row + 1] = c;
}

template <int G>
__global__ __launch_bounds__(256) void k_spgemm_expand(int64_t n, int wcap, const int32_t* rlo,
                                                      const int32_t* rwords,
                                                      const int64_t* wincl,
                                                      const uint32_t* wbuf, const int64_t* crp,
                                                      int32_t* ccol) {
  constexpr int NG = 256 / G, KW = 8;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  const int64_t row = xcd_block(blockIdx.x, gridDim.x) * NG + g;
  if (row >= n) return;
  const int nw = rwords[row];
  if (nw == 0 || nw > wcap) return;
  const int32_t lo = rlo[row];
  const uint32_t* src = wbuf + (wincl[row] - nw);
  int32_t* out = ccol + crp[row];
  // KW * G consecutive words per step, KW loads per lane in flight (lane l
  // holds words l, l + G, ...); each group of G words then places its set
  // bits by a scan of the popcounts over the group
  int run = 0;
  for (int t0 = 0; t0 < nw; t0 += KW * G) {
    uint32_t wv[KW];
#pragma unroll
    for (int k = 0; k < KW; k++) {
      const int t = t0 + k * G + lane;
      wv[k] = t < nw ? src[t] : 0u;
    }
#pragma unroll
    for (int k = 0; k < KW; k++) {
      const int t = t0 + k * G + lane;
      uint32_t m = wv[k];
      const int c = __popc(m);
      int incl = c;
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const int o = __shfl_up(incl, d, G);
        if (lane >= d) incl += o;
      }
      int p = run + incl - c;
      while (m) {
        const int b = __builtin_ctz(m);
        m &= m - 1u;
        out[p++] = lo + 32 * t + b;
      }
      run += __shfl(incl, G - 1, G);
    }
  }
}

__global__ void k_bounds_summary(const int64_t* wincl, int64_t n, const int* lerr,
                                 const unsigned long long* wmax, int64_t* out) {
  if (threadIdx.x == 0) {
    out[0] = n ? wincl[n - 1] : 0;
    out[1] = lerr[1];
    out[2] = (int64_t)*wmax;
  }
}

// the bounds kernel, and the bitmap kernel's MODE 2, with GQ lanes per row
template <int GQ>
static void launch_stored_q(int64_t n, const CsrView& A, const CsrView& B, int wcap,
                            int32_t* rlo, int32_t* rwords, int64_t* wcnt, int32_t* ovf, int* novf,
                            int wlds, uint32_t* wbuf, int64_t* cnt, int which, hipStream_t s) {
  constexpr int NG = 256 / GQ;
  if (which == 0) {
    k_spgemm_bounds<GQ><<<nblocks(n, NG), 256, 0, s>>>(n, A.rowptr, A.col, B.rowptr, B.col,
                                                       wcap, rlo, rwords, wcnt, ovf, novf);
  } else {
    allow_lds((const void*)k_spgemm_bits<GQ, 2>);
    k_spgemm_bits<GQ, 2><<<nblocks(n, NG), 256, (size_t)NG * wlds * sizeof(uint32_t), s>>>(
        n, A.rowptr, A.col, B.rowptr, B.col, wlds, wcap, rlo, rwords, wcnt, wbuf, cnt);
  }
}

static void stored_q_dispatch(int gq, int64_t n, const CsrView& A, const CsrView& B, int wcap,
                              int32_t* rlo, int32_t* rwords, int64_t* wcnt, int32_t* ovf,
                              int* novf, int wlds, uint32_t* wbuf, int64_t* cnt, int which,
                              hipStream_t s) {
  switch (gq) {
    case 4: launch_stored_q<4>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, which, s); break;
    case 8: launch_stored_q<8>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, which, s); break;
    case 16: launch_stored_q<16>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, which, s); break;
    case 32: launch_stored_q<32>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, which, s); break;
    default: launch_stored_q<64>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, which, s); break;
  }
}

template <int G>
static void launch_stored(int64_t n, const CsrView& A, const CsrView& B, int wcap, int32_t* rlo,
                          int32_t* rwords, int64_t* wcnt, int32_t* ovf, int* novf, int wlds,
                          uint32_t* wbuf, int64_t* cnt, const int64_t* crp, int32_t* ccol,
                          int which, int64_t wtotal, hipStream_t s) {
  // (long rows of A over B rows of a few dozen entries: flattened loads,
  // measured faster there than a lane walking each row; short B rows: four
  // A entries per lane, MODE 2; elsewhere the walk)
  const double avg_a = A.nrows ? (double)A.nnz / (double)A.nrows : 0.0;
  const double avg_b = B.nrows ? (double)B.nnz / (double)B.nrows : 0.0;
  const bool flat = avg_a >= 256.0 && avg_b >= 24.0 && avg_b < 64.0;
  const bool batched = !flat && avg_b <= 16.0;   // MODE 2
  constexpr int NG = 256 / G;
  // the unrolled kernels keep four entries per lane in flight: a quarter of
  // the lanes per row, more rows per wave, where that still leaves some 2048
  // waves to hide the latency (measured slower below that) and, for the
  // bitmaps of MODE 2, the block's bitmaps within the 32 KiB of LDS the walk
  // uses (more cuts the occupancy: measured slower)
  const int gq = G / 4 < 4 ? 4 : G / 4;
  const bool many = (double)n * gq / 64.0 >= 2048.0;
  const bool fits = (size_t)(256 / gq) * wlds * sizeof(uint32_t) <= 32 * 1024;
  // few rows of many products: several groups per row, up to about 2048
  // groups in all, each with at least 8 products per lane (the latency of
  // a lone group walking a long row is what bounds such a launch); where
  // a slice is too short to give each lane two A entries to walk, B rows of
  // two dozen entries or more are flattened over the lanes instead
  // (measured: the walk is faster for long slices, the flattened loads for
  // short ones)
  int nsl = 1;
  if (which == 1 && !many && n > 0) {
    const double want = std::ceil(2048.0 / (double)n);
    const double most = std::min(std::floor(avg_a * avg_b / (8.0 * G)), std::floor(avg_a));
    nsl = (int)std::max(1.0, std::min(std::min(want, most), 64.0));
  }
  const bool flat_sl = flat || (avg_a / nsl < 2.0 * G && avg_b >= 24.0);
  if (which == 0 && many) {
    stored_q_dispatch(gq, n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, 0, nullptr, nullptr, 0, s);
  } else if (which == 0) {
    k_spgemm_bounds<G><<<nblocks(n, NG), 256, 0, s>>>(n, A.rowptr, A.col, B.rowptr, B.col, wcap,
                                                      rlo, rwords, wcnt, ovf, novf);
  } else if (which == 1 && batched && many && fits) {
    stored_q_dispatch(gq, n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, 1, s);
  } else if (which == 1 && nsl > 1) {
    // few rows: nsl groups per row OR into the zeroed words, then the counts
    const size_t lds = (size_t)NG * wlds * sizeof(uint32_t);
    HIP_OK(hipMemsetAsync(wbuf, 0, (size_t)wtotal * sizeof(uint32_t), s));
    const int64_t ngr = n * nsl;
    if (flat_sl) {
      allow_lds((const void*)k_spgemm_bits<G, 1>);
      k_spgemm_bits<G, 1><<<nblocks(ngr, NG), 256, lds, s>>>(
          n, A.rowptr, A.col, B.rowptr, B.col, wlds, wcap, rlo, rwords, wcnt, wbuf, cnt, nsl);
    } else {
      allow_lds((const void*)k_spgemm_bits<G, 0>);
      k_spgemm_bits<G, 0><<<nblocks(ngr, NG), 256, lds, s>>>(
          n, A.rowptr, A.col, B.rowptr, B.col, wlds, wcap, rlo, rwords, wcnt, wbuf, cnt, nsl);
    }
    k_spgemm_bits_count<G><<<nblocks(n, NG), 256, 0, s>>>(n, wcap, rwords, wcnt, wbuf, cnt);
  } else if (which == 1) {
    const size_t lds = (size_t)NG * wlds * sizeof(uint32_t);
    if (flat) {
      allow_lds((const void*)k_spgemm_bits<G, 1>);
      k_spgemm_bits<G, 1><<<nblocks(n, NG), 256, lds, s>>>(
          n, A.rowptr, A.col, B.rowptr, B.col, wlds, wcap, rlo, rwords, wcnt, wbuf, cnt);
    } else {
      allow_lds((const void*)k_spgemm_bits<G, 0>);
      k_spgemm_bits<G, 0><<<nblocks(n, NG), 256, lds, s>>>(
          n, A.rowptr, A.col, B.rowptr, B.col, wlds, wcap, rlo, rwords, wcnt, wbuf, cnt);
    }
  } else if ((double)n * 16 / 64.0 >= 2048.0) {
    // (the expansion reads words only: 16 lanes per row whatever G, given
    // rows enough to fill the machine)
    k_spgemm_expand<16><<<nblocks(n, 16), 256, 0, s>>>(n, wcap, rlo, rwords, wcnt, wbuf, crp,
                                                       ccol);
  } else {
    k_spgemm_expand<G><<<nblocks(n, NG), 256, 0, s>>>(n, wcap, rlo, rwords, wcnt, wbuf, crp,
                                                      ccol);
  }
}

static void stored_dispatch(int g, int64_t n, const CsrView& A, const CsrView& B, int wcap,
                            int32_t* rlo, int32_t* rwords, int64_t* wcnt, int32_t* ovf, int* novf,
                            int wlds, uint32_t* wbuf, int64_t* cnt, const int64_t* crp,
                            int32_t* ccol, int which, int64_t wtotal, hipStream_t s) {
  switch (g) {
    case 4: launch_stored<4>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, crp, ccol, which, wtotal, s); break;
    case 8: launch_stored<8>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, crp, ccol, which, wtotal, s); break;
    case 16: launch_stored<16>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, crp, ccol, which, wtotal, s); break;
    case 32: launch_stored<32>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, crp, ccol, which, wtotal, s); break;
    default: launch_stored<64>(n, A, B, wcap, rlo, rwords, wcnt, ovf, novf, wlds, wbuf, cnt, crp, ccol, which, wtotal, s); break;
  }
}

// hash kernels for a list of rows (those outside the window kernel's reach)
template <int G>
static void launch_sym_rows(const int32_t* rows, int64_t nrows, const CsrView& A,
                            const CsrView& B, int hcap, int64_t* cnt, const int64_t* crp,
                            int32_t* ccol, int32_t* ovf, int* novf, int* derr, hipStream_t s) {
  if (nrows) launch_sym<G, 256>(rows, nrows, A, B, hcap, cnt, crp, ccol, ovf, novf, derr, s);
}

void spgemm_symbolic(const CsrView& A, const CsrView& B, Csr& C, SpgemmPlan& plan,
                     hipStream_t s, Arena& ar, int* derr, bool split, Scratch* scratch) {
  if (A.ncols != B.nrows) throw Error(EMIN_ERR_SHAPE, "spgemm: inner dimensions differ");
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.rowptr = ar.alloc<int64_t>(C.nrows + 1);
  HIP_OK(hipMemsetAsync(C.rowptr, 0, sizeof(int64_t) * (C.nrows + 1), s));
  const double avg_a = A.nrows ? (double)A.nnz / (double)A.nrows : 1.0;
  const int g = pick_g(avg_a);
  const int NG = 256 / g;
  // window bitmap per group: up to 32 KiB per block
  const int wcap = (int)std::min<int64_t>(4096, (32 * 1024 / 4) / NG);
  const int big = 16384;  // hash table of one 64-lane group, 96 KiB of LDS
  int* lerr = ar.alloc<int>(4);   // error, wide rows, hash overflow, fill overflow
  int32_t* rwords = ar.alloc<int32_t>(A.nrows);   // words spanned by each output row
  int32_t* ovf = ar.alloc<int32_t>(A.nrows);    // rows wider than the window
  int32_t* ovf2 = ar.alloc<int32_t>(A.nrows);   // of those, rows the hash table cannot hold
  HIP_OK(hipMemsetAsync(lerr, 0, 4 * sizeof(int), s));
  int hl[4];
  int nwide = 0;
  // stored bitmaps: the windows first, then one pass that forms the products
  bool stored = false;
  int32_t* rlo = nullptr;
  int64_t* wincl = nullptr;
  uint32_t* wbuf = nullptr;
  if (scratch && A.nrows) {
    rlo = ar.alloc<int32_t>(A.nrows);
    wincl = ar.alloc<int64_t>(A.nrows);
    unsigned long long* wmax = ar.alloc<unsigned long long>(1);
    int64_t* bs = ar.alloc<int64_t>(3);
    HIP_OK(hipMemsetAsync(wmax, 0, sizeof(unsigned long long), s));
    stored_dispatch(g, A.nrows, A, B, wcap, rlo, rwords, wincl, ovf, lerr + 1, 0, nullptr,
                    nullptr, nullptr, nullptr, 0, 0, s);
    k_wcnt_max<<<nblocks(A.nrows, 1024), 256, 0, s>>>(wincl, A.nrows, wmax);
    scan_inclusive(wincl, A.nrows, s, ar);
    k_bounds_summary<<<1, 64, 0, s>>>(wincl, A.nrows, lerr, wmax, bs);
    int64_t hb[3];
    read_back(hb, bs, sizeof(hb), s);
    nwide = (int)hb[1];
    if ((size_t)hb[0] * sizeof(uint32_t) <= kStoredBitmapMax) {
      stored = true;
      wbuf = static_cast<uint32_t*>(scratch->get((size_t)(hb[0] > 0 ? hb[0] : 1) * sizeof(uint32_t)));
      const int wlds = (int)std::max<int64_t>(hb[2], 1);
      stored_dispatch(g, A.nrows, A, B, wcap, rlo, rwords, wincl, nullptr, nullptr, wlds, wbuf,
                      C.rowptr, nullptr, nullptr, 1, hb[0], s);
    } else {
      // too many words to keep: the two-pass form (which lists the wide rows again)
      HIP_OK(hipMemsetAsync(lerr + 1, 0, sizeof(int), s));
    }
  }
  if (!stored) {
    if (A.nrows)
      win_dispatch(g, A.nrows, A, B, wcap, C.rowptr, nullptr, nullptr, ovf, lerr + 1, rwords, s);
    read_back(hl, lerr, sizeof(hl), s);
    nwide = hl[1];
  }
  // table per group within ~48 KiB per block (keys + compacted copy)
  int hcap = 64;
  while ((size_t)NG * 3 * hcap * sizeof(int32_t) <= 48 * 1024 && hcap < 4096) hcap <<= 1;
  int nov = 0;
  if (nwide) {
    switch (g) {
      case 4: launch_sym_rows<4>(ovf, nwide, A, B, hcap, C.rowptr, nullptr, nullptr, ovf2, lerr + 2, lerr, s); break;
      case 8: launch_sym_rows<8>(ovf, nwide, A, B, hcap, C.rowptr, nullptr, nullptr, ovf2, lerr + 2, lerr, s); break;
      case 16: launch_sym_rows<16>(ovf, nwide, A, B, hcap, C.rowptr, nullptr, nullptr, ovf2, lerr + 2, lerr, s); break;
      case 32: launch_sym_rows<32>(ovf, nwide, A, B, hcap, C.rowptr, nullptr, nullptr, ovf2, lerr + 2, lerr, s); break;
      default: launch_sym_rows<64>(ovf, nwide, A, B, hcap, C.rowptr, nullptr, nullptr, ovf2, lerr + 2, lerr, s); break;
    }
    read_back(hl, lerr, sizeof(hl), s);
    nov = hl[2];
    if (nov) sym_big(ovf2, nov, A, B, big, C.rowptr, nullptr, nullptr, lerr, s);
  }
  // one read-back: output size, count-pass overflow, longest output row
  HIP_OK(hipMemsetAsync(C.rowptr, 0, sizeof(int64_t), s));
  scan_inclusive(C.rowptr + 1, C.nrows, s, ar);
  unsigned long long* mx = ar.alloc<unsigned long long>(5);
  int64_t* sm = ar.alloc<int64_t>(7);
  HIP_OK(hipMemsetAsync(mx, 0, 5 * sizeof(unsigned long long), s));
  if (C.nrows)
    k_sym_maxima<<<nblocks(C.nrows, 256), 256, 0, s>>>(
        C.rowptr, rwords, split ? A.rowptr : nullptr, A.rowptr, C.nrows, mx);
  k_sym_summary<<<1, 64, 0, s>>>(C.rowptr, C.nrows, lerr, mx, sm);
  int64_t hs[7];
  read_back(hs, sm, sizeof(hs), s);
  C.nnz = hs[0];
  if (hs[1]) throw Error(EMIN_ERR_CAPACITY, "spgemm: output row exceeds the LDS table");
  plan.max_row = hs[2];
  plan.max_words = hs[3];
  plan.ntasks = hs[4];
  plan.max_arow = hs[6];
  if (plan.ntasks) {
    // long rows: work items (row, chunk) and the offsets of their chunk sums
    const int64_t n = C.nrows;
    int64_t* ch = ar.alloc<int64_t>(n);
    int64_t* vals = ar.alloc<int64_t>(n);
    int32_t* trow = ar.alloc<int32_t>(plan.ntasks);
    int32_t* tchunk = ar.alloc<int32_t>(plan.ntasks);
    int64_t* poff = ar.alloc<int64_t>(n);
    k_split_counts<<<nblocks(n, 256), 256, 0, s>>>(C.rowptr, A.rowptr, n, ch, vals);
    scan_inclusive(ch, n, s, ar);
    scan_inclusive(vals, n, s, ar);
    k_split_fill<<<nblocks(n, 256), 256, 0, s>>>(C.rowptr, ch, vals, n, trow, tchunk, poff);
    plan.task_row = trow;
    plan.task_chunk = tchunk;
    plan.poff = poff;
    plan.part = ar.alloc<double>(hs[5]);
  }
  C.col = ar.alloc<int32_t>(C.nnz);
  C.val = ar.alloc<double>(C.nnz);
  // the window fill skips the wide rows; the hash kernels fill those (the
  // first hash fill skips the rows its table could not hold; the big table
  // does them)
  if (A.nrows && stored)
    stored_dispatch(g, A.nrows, A, B, wcap, rlo, rwords, wincl, nullptr, nullptr, 0, wbuf,
                    nullptr, C.rowptr, C.col, 2, 0, s);
  else if (A.nrows)
    win_dispatch(g, A.nrows, A, B, wcap, nullptr, C.rowptr, C.col, nullptr, nullptr, nullptr, s);
  if (nwide) {
    switch (g) {
      case 4: launch_sym_rows<4>(ovf, nwide, A, B, hcap, nullptr, C.rowptr, C.col, ovf2, lerr + 3, lerr, s); break;
      case 8: launch_sym_rows<8>(ovf, nwide, A, B, hcap, nullptr, C.rowptr, C.col, ovf2, lerr + 3, lerr, s); break;
      case 16: launch_sym_rows<16>(ovf, nwide, A, B, hcap, nullptr, C.rowptr, C.col, ovf2, lerr + 3, lerr, s); break;
      case 32: launch_sym_rows<32>(ovf, nwide, A, B, hcap, nullptr, C.rowptr, C.col, ovf2, lerr + 3, lerr, s); break;
      default: launch_sym_rows<64>(ovf, nwide, A, B, hcap, nullptr, C.rowptr, C.col, ovf2, lerr + 3, lerr, s); break;
    }
    if (nov) sym_big(ovf2, nov, A, B, big, nullptr, C.rowptr, C.col, lerr, s);
  }
  if (derr) k_defer_err<<<1, 64, 0, s>>>(lerr, derr);
  else if (d2h(lerr, s)) throw Error(EMIN_ERR_CAPACITY, "spgemm: fill pass overflow");
  const double avg_b = B.nrows ? (double)B.nnz / (double)B.nrows : 1.0;
  int gn = pick_g(avg_b);
  // long rows of A (hundreds of entries: B B^T, B (I (x) P), the coarse
  // levels) have long output rows with wide windows; twice the lanes halve
  // the groups, and so the LDS, of a block, and more waves stay resident
  // (measured: 1.1-1.8x on those products; shorter rows lose by it)
  if (avg_a >= 128.0 && gn < 64) gn <<= 1;
  // enough lanes per row that the longest output row fits the LDS budget
  while (gn < 64 && (size_t)(256 / gn) * plan.max_row * 12 > 96 * 1024) gn <<= 1;
  plan.g_num = gn;
}

// Numeric product for few output rows: each row's entries are cut into S
// slices of consecutive columns, one group of G lanes per (row, slice), so
// that rows too few to fill the device still keep it busy.  The group takes
// the row's A entries in ascending order, G at a time: lane q finds where
// B's row of entry q meets the slice's column range (two binary searches);
// then, entry by entry, the lanes add that part's products into the slice's
// accumulators (slot of a column by binary search over the slice's sorted
// columns in LDS).  The columns of one B row are distinct, so every c_ij
// still receives its products in ascending order of A's row, each product
// and each sum rounded separately.
template <int G, class TV, class TO>
__global__ __launch_bounds__(256) void k_spgemm_num_slices(const int64_t* arp,
                                                          const int32_t* acol, const TV* aval,
                                                          const int64_t* brp,
                                                          const int32_t* bcol, const TV* bval,
                                                          const int64_t* crp,
                                                          const int32_t* ccol, TO* cval,
                                                          int64_t n, int S, int L) {
  extern __shared__ uint32_t lds_words[];
  constexpr int NG = 256 / G;
  const int g = threadIdx.x / G, lane = threadIdx.x % G;
  int32_t* scol = reinterpret_cast<int32_t*>(lds_words) + (size_t)g * L;
  TV* acc = reinterpret_cast<TV*>(lds_words + (size_t)NG * L) + (size_t)g * L;
  const int64_t item = (int64_t)blockIdx.x * NG + g;
  const int64_t row = item / S;
  const int t = (int)(item % S);
  if (row >= n) return;
  const int64_t c0 = crp[row];
  const int nc = (int)(crp[row + 1] - c0);
  const int len = (nc + S - 1) / S;
  const int s0 = t * len, s1 = s0 + len < nc ? s0 + len : nc;
  if (s0 >= s1) return;
  const int ns = s1 - s0;
  for (int q = lane; q < ns; q += G) {
    scol[q] = ccol[c0 + s0 + q];
    acc[q] = TV(0);
  }
  group_sync_lds<G>();
  const int32_t j0 = scol[0], j1 = scol[ns - 1];
  const int64_t ea = arp[row], eb = arp[row + 1];
  for (int64_t e0 = ea; e0 < eb; e0 += G) {
    int64_t p0 = 0;
    int pl = 0;
    TV av = TV(0);
    if (e0 + lane < eb) {
      const int32_t k = acol[e0 + lane];
      av = aval[e0 + lane];
      const int64_t b0 = brp[k], b1 = brp[k + 1];
      int64_t lo = b0, hi = b1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (bcol[mid] < j0) lo = mid + 1; else hi = mid;
      }
      p0 = lo;
      hi = b1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (bcol[mid] <= j1) lo = mid + 1; else hi = mid;
      }
      pl = (int)(lo - p0);
    }
    const int cnt = (int)((eb - e0) < G ? (eb - e0) : G);
    auto slot = [&](int32_t j) {
      int lo = 0, hi = ns;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (scol[mid] < j) lo = mid + 1; else hi = mid;
      }
      return lo;
    };
    // SU entries at a time: the first G entries of each one's B range are
    // loaded together, then added in the entries' order (the rest of a range
    // longer than the group follows its entry's first part)
    constexpr int SU = 8;
    for (int q0 = 0; q0 < cnt; q0 += SU) {
      int64_t pq[SU];
      int lq[SU], sl[SU];
      TV aq[SU], pr[SU];
#pragma unroll
      for (int u = 0; u < SU; u++) {
        const int q = q0 + u;
        pq[u] = __shfl(p0, q, G);
        lq[u] = q < cnt ? __shfl(pl, q, G) : 0;
        aq[u] = __shfl(av, q, G);
        int32_t j = -1;
        TV b = TV(0);
        if (lane < lq[u]) {
          j = bcol[pq[u] + lane];
          b = bval[pq[u] + lane];
        }
        sl[u] = j;
        pr[u] = b;
      }
#pragma unroll
      for (int u = 0; u < SU; u++) sl[u] = sl[u] >= 0 ? slot(sl[u]) : -1;
#pragma unroll
      for (int u = 0; u < SU; u++) {
        if (sl[u] >= 0) acc_add(acc, sl[u], aq[u] * pr[u]);
        for (int o = G + lane; o < lq[u]; o += G) {
          const int32_t j = bcol[pq[u] + o];
          const TV b = bval[pq[u] + o];
          acc_add(acc, slot(j), aq[u] * b);
        }
        acc_order<TV>();
      }
    }
  }
  group_sync_lds<G>();
  for (int q = lane; q < ns; q += G) cval[c0 + s0 + q] = (TO)acc[q];
}

// products with at most this many rows take the slice kernel (when their
// rows are long enough to cut)
constexpr int64_t SLICE_MAX_ROWS = 4096;

template <class TV, class TO>
static bool numeric_slices(const CsrView& A, const TV* aval, const CsrView& B, const TV* bval,
                           const Csr& C, TO* cval, const SpgemmPlan& plan, hipStream_t s) {
  if (A.nrows > SLICE_MAX_ROWS || A.nrows == 0 || plan.max_row < 64) return false;
  // every group walks its row's whole A list, so A's rows must be short, and
  // an average B row must still put several entries into each slice
  const double avg_a = (double)A.nnz / (double)A.nrows;
  const double avg_b = B.nrows ? (double)B.nnz / (double)B.nrows : 0.0;
  if (avg_a > 512.0) return false;
  constexpr int G = 32, NG = 256 / G;
  // about 8K groups over the device, slices of at least 16 entries and at
  // least 8 entries of an average B row, and the slice columns and
  // accumulators of a block within 64 KiB
  int64_t S = (8192 + A.nrows - 1) / A.nrows;
  S = std::min<int64_t>(S, plan.max_row / 16);
  S = std::min<int64_t>(S, (int64_t)(avg_b / 8.0));
  if (S < 2) return false;
  int64_t L = (plan.max_row + S - 1) / S;
  while ((size_t)NG * L * (4 + sizeof(TV)) > 64 * 1024) {
    S++;
    L = (plan.max_row + S - 1) / S;
  }
  L = (L + 1) & ~int64_t(1);   // (keeps the accumulators 8-byte aligned)
  const size_t lds = (size_t)NG * L * (4 + sizeof(TV));
  allow_lds((const void*)k_spgemm_num_slices<G, TV, TO>);
  const int64_t items = A.nrows * S;
  k_spgemm_num_slices<G, TV, TO><<<nblocks(items, NG), 256, lds, s>>>(
      A.rowptr, A.col, aval, B.rowptr, B.col, bval, C.rowptr, C.col, cval, A.nrows, (int)S,
      (int)L);
  return true;
}

template <int G, class TV, class TO>
static void launch_num(const CsrView& A, const TV* aval, const CsrView& B, const TV* bval,
                       const Csr& C, TO* cval, int cap, int iw, const SpgemmPlan& plan,
                       hipStream_t s) {
  constexpr int NG = 256 / G;
  const size_t lds = (size_t)NG * ((size_t)iw * sizeof(uint32_t) + cap * sizeof(TV));
  allow_lds((const void*)k_spgemm_num<G, TV, TO>);
  SplitArgsT<TV> rows_only;
  rows_only.poff = plan.ntasks ? plan.poff : nullptr;
  k_spgemm_num<G, TV, TO><<<nblocks(A.nrows, NG), 256, lds, s>>>(
      A.rowptr, A.col, aval, B.rowptr, B.col, bval, C.rowptr, C.col, cval, A.nrows, cap, iw,
      rows_only);
  if (plan.ntasks) {
    SplitArgsT<TV> sp;
    sp.trow = plan.task_row;
    sp.tchunk = plan.task_chunk;
    sp.poff = plan.poff;
    sp.part = reinterpret_cast<TV*>(plan.part);
    sp.ntasks = plan.ntasks;
    k_spgemm_num<G, TV, TO><<<nblocks(plan.ntasks, NG), 256, lds, s>>>(
        A.rowptr, A.col, aval, B.rowptr, B.col, bval, C.rowptr, C.col, cval, A.nrows, cap, iw,
        sp);
    k_spgemm_combine<TV, TO><<<nblocks(plan.ntasks, 4), 256, 0, s>>>(A.rowptr, C.rowptr, sp, cval);
  }
}

template <class TV, class TO>
static void numeric_any(const CsrView& A, const TV* aval, const CsrView& B, const TV* bval,
                        const Csr& C, TO* cval, const SpgemmPlan& plan, hipStream_t s) {
  if (A.nrows == 0 || C.nnz == 0) return;
  prof::Scope ps(s, EMIN_PROF_SPGEMM,
                 (4.0 + sizeof(TV)) * (double)(A.nnz + B.nnz + C.nnz) + 16.0 * (double)A.nrows);
  if (numeric_slices<TV, TO>(A, aval, B, bval, C, cval, plan, s)) return;
  const int g = plan.g_num;
  const int NG = 256 / g;
  // LDS: accumulators of the longest row (within ~96 KiB per block), and an
  // index of iw words per row: enough for the two-level index of every window
  // row, the flat window where ~40 KiB per block allow it, never less than
  // the sorted columns, and within 152 KiB per block in all
  int cap = (int)((96 * 1024) / (NG * (sizeof(TV) + sizeof(int32_t))));
  if (cap > plan.max_row) cap = (int)plan.max_row;
  if (cap < 1) cap = 1;
  const int64_t mw = plan.max_words;
  const int64_t two_level = 2 * ((mw + 31) / 32 + cap);
  const int64_t flat = std::min<int64_t>(2 * mw, (40 * 1024 / NG - (int64_t)cap * sizeof(TV)) / 4);
  const int64_t most = (152 * 1024 / NG - (int64_t)cap * sizeof(TV)) / 4;
  // (the two-level room only where some window row misses the flat one)
  int64_t iw = std::min(flat >= 2 * mw ? flat : std::max(two_level, flat), most);
  iw = std::max<int64_t>(iw, cap);
  iw = (iw + 1) & ~int64_t(1);
  switch (g) {
    case 4: launch_num<4>(A, aval, B, bval, C, cval, cap, (int)iw, plan, s); break;
    case 8: launch_num<8>(A, aval, B, bval, C, cval, cap, (int)iw, plan, s); break;
    case 16: launch_num<16>(A, aval, B, bval, C, cval, cap, (int)iw, plan, s); break;
    case 32: launch_num<32>(A, aval, B, bval, C, cval, cap, (int)iw, plan, s); break;
    default: launch_num<64>(A, aval, B, bval, C, cval, cap, (int)iw, plan, s); break;
  }
  if (plan.max_row > cap)
    k_spgemm_num_long<TV, TO><<<nblocks(A.nrows, 64), 64, 0, s>>>(
        A.rowptr, A.col, aval, B.rowptr, B.col, bval, C.rowptr, C.col, cval, A.nrows, cap);
}

// C = A A^T by dot products (see spgemm_numeric_aat): one wave per output row
// i; row i of A staged in LDS (its values, and a flat or two-level bitmap of
// its columns giving the position of column k, as in k_spgemm_num); lane t
// takes the output entries t, t + 64, ...: c_ij walks row j of A in column
// order and adds a_ik * a_jk for the columns present in row i.
__global__ __launch_bounds__(64) void k_spgemm_aat(const int64_t* arp, const int32_t* acol,
                                                  const double* aval, const int64_t* crp,
                                                  const int32_t* ccol, double* cval, int64_t n,
                                                  int iw) {
  extern __shared__ uint32_t lds_words[];
  uint32_t* idx = lds_words;                                  // iw words (iw even)
  double* av = reinterpret_cast<double*>(lds_words + iw);     // row i's values
  const int lane = threadIdx.x;
  const int64_t row = blockIdx.x;
  if (row >= n) return;
  const int64_t c0 = crp[row];
  const int nc = (int)(crp[row + 1] - c0);
  const int64_t a0 = arp[row];
  const int la = (int)(arp[row + 1] - a0);
  if (nc == 0) return;
  if (la == 0) {
    for (int t = lane; t < nc; t += 64) cval[c0 + t] = 0.0;
    return;
  }
  const int32_t klo = acol[a0], khi = acol[a0 + la - 1];
  const int64_t nw = (((int64_t)khi - klo) >> 5) + 1, nw1 = (nw + 31) >> 5;
  const bool flat = 2 * nw <= iw;   // else two-level (sized to fit by the host)
  uint32_t* cw = idx + 2 * nw1;
  for (int t = lane; t < la; t += 64) av[t] = aval[a0 + t];
  if (flat) {
    for (int64_t t = lane; t < nw; t += 64) idx[2 * t] = 0u;
  } else {
    for (int64_t t = lane; t < nw1; t += 64) idx[2 * t] = 0u;
    for (int t = lane; t < la; t += 64) cw[2 * t] = 0u;
  }
  group_sync_lds<64>();
  if (flat) {
    for (int t = lane; t < la; t += 64) {
      const int r = acol[a0 + t] - klo;
      const int w = r >> 5;
      atomicOr(&idx[2 * w], 1u << (r & 31));
      if (t == 0 || ((acol[a0 + t - 1] - klo) >> 5) != w) idx[2 * w + 1] = (uint32_t)t;
    }
  } else {
    for (int t = lane; t < la; t += 64) {
      const int w = (acol[a0 + t] - klo) >> 5;
      atomicOr(&idx[2 * (w >> 5)], 1u << (w & 31));
    }
    group_sync_lds<64>();
    int run = 0;
    for (int64_t s0 = 0; s0 < nw1; s0 += 64) {
      const int64_t sw = s0 + lane;
      const int c = sw < nw1 ? __popc(idx[2 * sw]) : 0;
      int incl = c;
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) {
        const int o = __shfl_up(incl, m, 64);
        if (lane >= m) incl += o;
      }
      if (sw < nw1) idx[2 * sw + 1] = (uint32_t)(run + incl - c);
      run += __shfl(incl, 63, 64);
    }
    group_sync_lds<64>();
    for (int t = lane; t < la; t += 64) {
      const int r = acol[a0 + t] - klo;
      const int w = r >> 5, sw = w >> 5;
      const int d = (int)idx[2 * sw + 1] + __popc(idx[2 * sw] & ((1u << (w & 31)) - 1u));
      atomicOr(&cw[2 * d], 1u << (r & 31));
      if (t == 0 || ((acol[a0 + t - 1] - klo) >> 5) != w) cw[2 * d + 1] = (uint32_t)t;
    }
  }
  group_sync_lds<64>();
  // position of column k in row i, or -1
  auto pos_of = [&](int32_t k) -> int {
    if (k < klo || k > khi) return -1;
    const int r = k - klo, w = r >> 5;
    const uint32_t bit = 1u << (r & 31);
    uint2 e;
    if (flat) {
      e = *reinterpret_cast<const uint2*>(idx + 2 * w);
    } else {
      const uint2 e1 = *reinterpret_cast<const uint2*>(idx + 2 * (w >> 5));
      const uint32_t wb = 1u << (w & 31);
      if (!(e1.x & wb)) return -1;
      const int d = (int)e1.y + __popc(e1.x & (wb - 1u));
      e = *reinterpret_cast<const uint2*>(cw + 2 * d);
    }
    if (!(e.x & bit)) return -1;
    return (int)e.y + __popc(e.x & (bit - 1u));
  };
  for (int t = lane; t < nc; t += 64) {
    const int32_t j = ccol[c0 + t];
    const int64_t b0 = arp[j], b1 = arp[j + 1];
    double acc = 0.0;
    int64_t e = b0;
    // (sixteen entries' loads in flight per lane: a row j of a coarse B runs
    // to a thousand entries, walked one lane per output)
    constexpr int U = 16;
    for (; e + U <= b1; e += U) {
      int32_t k[U];
      double v[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        k[u] = acol[e + u];
        v[u] = aval[e + u];
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int p = pos_of(k[u]);
        if (p >= 0) acc = acc + av[p] * v[u];
      }
    }
    for (; e < b1; e++) {
      const int p = pos_of(acol[e]);
      if (p >= 0) acc = acc + av[p] * aval[e];
    }
    cval[c0 + t] = acc;
  }
}

void spgemm_numeric_aat(const CsrView& A, const CsrView& At, const Csr& C, const SpgemmPlan& plan,
                        hipStream_t s) {
  // index words for the two-level form of the longest row, the flat one
  // where it fits in the same room; with the values, within ~150 KiB
  const int64_t nw1 = ((A.ncols + 31) / 32 + 31) / 32;
  int64_t iw = 2 * (nw1 + plan.max_arow);
  iw = (iw + 1) & ~int64_t(1);
  const size_t lds = (size_t)iw * 4 + (size_t)plan.max_arow * 8;
  // (measured: with more than a few hundred rows the row-parallel kernel is
  // faster; the dot products pay off where few long rows leave it idle)
  if (plan.max_arow <= SPGEMM_SPLIT || A.nrows > 256 || lds > 150 * 1024 || A.nrows == 0 ||
      C.nnz == 0) {
    spgemm_numeric(A, At, C, plan, s);
    return;
  }
  prof::Scope ps(s, EMIN_PROF_SPGEMM, 12.0 * (double)(A.nnz + At.nnz + C.nnz));
  allow_lds((const void*)k_spgemm_aat);
  k_spgemm_aat<<<(unsigned)A.nrows, 64, lds, s>>>(A.rowptr, A.col, A.val, C.rowptr, C.col, C.val,
                                                  A.nrows, (int)iw);
}

void spgemm_numeric(const CsrView& A, const CsrView& B, const Csr& C, const SpgemmPlan& plan,
                    hipStream_t s) {
  numeric_any<double, double>(A, A.val, B, B.val, C, C.val, plan, s);
}

void spgemm_numeric_f32(const CsrView& A, const float* aval, const CsrView& B, const float* bval,
                        const Csr& C, float* cval32, double* cval64, const SpgemmPlan& plan,
                        hipStream_t s) {
  if (cval64) numeric_any<float, double>(A, aval, B, bval, C, cval64, plan, s);
  else numeric_any<float, float>(A, aval, B, bval, C, cval32, plan, s);
}

__global__ void k_gather_f(const float* in, const int32_t* src, float* out, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = in[src[p]];
}

void gather_values_f(const float* in, const int32_t* src, float* out, int64_t n, hipStream_t s) {
  if (n) k_gather_f<<<nblocks(n, 256), 256, 0, s>>>(in, src, out, n);
}

// ---------------------------------------------------------------------------
// eq. (e:filtering): keep off-diagonal a_ij iff a_ij^2 > tau1^2 |a_ii a_jj|;
// dropped entries lumped into the diagonal in ascending column order.
// ---------------------------------------------------------------------------
__global__ void k_diag(const int64_t* rp, const int32_t* col, const double* val, int64_t n,
                       double* d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  int64_t lo = rp[i], hi = rp[i + 1];
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (col[mid] < i) lo = mid + 1; else hi = mid;
  }
  if (lo < rp[i + 1] && col[lo] == i) v = val[lo];
  d[i] = v;
}

void diag_of(const CsrView& A, double* d, hipStream_t s) {
  if (A.nrows) k_diag<<<nblocks(A.nrows, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, A.nrows, d);
}



void filter_symbolic(const CsrView& A, double tau1, const double* d, uint8_t* keep, Csr& At,
                     hipStream_t s, Arena& ar, uint8_t* dir) {
  At.nrows = At.ncols = A.nrows;
  At.rowptr = ar.alloc<int64_t>(A.nrows + 1);
  const double t2 = tau1 * tau1;
  if (A.nrows)
    ROWS_DISPATCH(lanes_for(A), k_filter_count_g, A.nrows, s, A.rowptr, A.col, A.val, A.nrows, t2,
                  d, keep, At.rowptr, dir);
  At.nnz = rowptr_from_counts(At.rowptr, A.nrows, s, ar);
  At.col = ar.alloc<int32_t>(At.nnz);
  At.val = ar.alloc<double>(At.nnz);
  if (A.nrows)
    ROWS_DISPATCH(lanes_for(A), k_filter_fill_g, A.nrows, s, A.rowptr, A.col, A.val, A.nrows, keep,
                  d, At.rowptr, At.col, At.val);
}

void filter_numeric(const CsrView& A, const uint8_t* keep, const double* d, const Csr& At,
                    hipStream_t s) {
  if (A.nrows)
    ROWS_DISPATCH(lanes_for(A), k_filter_fill_g, A.nrows, s, A.rowptr, A.col, A.val, A.nrows, keep,
                  d, At.rowptr, (int32_t*)nullptr, At.val);
}

// ---------------------------------------------------------------------------
// M = (A + A^T)/2 on the union pattern, m_ij = (a_ij + a_ji)*0.5
// ---------------------------------------------------------------------------
// Row i of the union pattern: a merge of A's row i with row i of A^T (the
// transposed entries carry their source position in A), one thread per row;
// ia/ib give each union entry's position in A for a_ij and a_ji (-1: absent).
// UB consecutive rows per block, their entries of A and of the transpose
// first staged in LDS with coalesced loads (a per-thread walk over global
// memory is bound by its dependent, scattered loads); a block whose rows hold
// more than UCAP entries of either merges from global memory instead.
constexpr int UB = 128, UCAP = 4096;
__global__ __launch_bounds__(UB) void k_union_blk(const int64_t* arp, const int32_t* acol,
                                                  const int64_t* trp, const int32_t* tcol,
                                                  const int32_t* tsrc, int64_t n, int64_t* cnt,
                                                  const int64_t* mrp, int32_t* mcol, int32_t* ia,
                                                  int32_t* ib) {
  __shared__ int32_t sa[UCAP], st[UCAP], ss[UCAP];
  const int64_t i0 = (int64_t)blockIdx.x * UB;
  const int64_t i1 = i0 + UB < n ? i0 + UB : n;
  const int64_t ba = arp[i0], bt = trp[i0];
  const int64_t na = arp[i1] - ba, nt = trp[i1] - bt;
  const bool staged = na <= UCAP && nt <= UCAP;   // uniform over the block
  if (staged) {
    for (int64_t t = threadIdx.x; t < na; t += UB) sa[t] = acol[ba + t];
    for (int64_t t = threadIdx.x; t < nt; t += UB) {
      st[t] = tcol[bt + t];
      ss[t] = tsrc[bt + t];
    }
  }
  __syncthreads();
  const int64_t i = i0 + threadIdx.x;
  if (i >= n) return;
  int64_t a = arp[i], ae = arp[i + 1], b = trp[i], be = trp[i + 1];
  int64_t p = mrp ? mrp[i] : 0, c = 0;
  if (staged) {
    int la = (int)(a - ba);
    const int lae = (int)(ae - ba);
    int lb = (int)(b - bt);
    const int lbe = (int)(be - bt);
    while (la < lae || lb < lbe) {
      int32_t j, x = -1, y = -1;
      const int32_t ca = la < lae ? sa[la] : INT32_MAX;
      const int32_t ct = lb < lbe ? st[lb] : INT32_MAX;
      if (ca < ct) { j = ca; x = (int32_t)(ba + la); la++; }
      else if (ct < ca) { j = ct; y = ss[lb]; lb++; }
      else { j = ca; x = (int32_t)(ba + la); y = ss[lb]; la++; lb++; }
      if (mcol) { mcol[p + c] = j; ia[p + c] = x; ib[p + c] = y; }
      c++;
    }
  } else {
    while (a < ae || b < be) {
      int32_t j;
      int32_t x = -1, y = -1;
      if (b >= be || (a < ae && acol[a] < tcol[b])) { j = acol[a]; x = (int32_t)a; a++; }
      else if (a >= ae || tcol[b] < acol[a]) { j = tcol[b]; y = tsrc[b]; b++; }
      else { j = acol[a]; x = (int32_t)a; y = tsrc[b]; a++; b++; }
      if (mcol) { mcol[p + c] = j; ia[p + c] = x; ib[p + c] = y; }
      c++;
    }
  }
  if (cnt) cnt[i + 1] = c;
}

__global__ void k_sym_vals(const double* aval, const int32_t* ia, const int32_t* ib, double* mval,
                           int64_t nnz) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const double x = ia[e] >= 0 ? aval[ia[e]] : 0.0;
  const double y = ib[e] >= 0 ? aval[ib[e]] : 0.0;
  mval[e] = (x + y) * 0.5;
}

void symmetrize_symbolic(const Csr& A, Csr& M, int32_t*& ia, int32_t*& ib, hipStream_t s,
                         Arena& ar) {
  Csr T;
  int32_t* tsrc = nullptr;
  transpose_pattern(view(A), T, tsrc, s, ar);
  M.nrows = M.ncols = A.nrows;
  M.rowptr = ar.alloc<int64_t>(A.nrows + 1);
  if (A.nrows)
    k_union_blk<<<nblocks(A.nrows, UB), UB, 0, s>>>(A.rowptr, A.col, T.rowptr, T.col, tsrc,
                                                     A.nrows, M.rowptr, nullptr, nullptr,
                                                     nullptr, nullptr);
  M.nnz = rowptr_from_counts(M.rowptr, A.nrows, s, ar);
  M.col = ar.alloc<int32_t>(M.nnz);
  M.val = ar.alloc<double>(M.nnz);
  ia = ar.alloc<int32_t>(M.nnz);
  ib = ar.alloc<int32_t>(M.nnz);
  if (A.nrows)
    k_union_blk<<<nblocks(A.nrows, UB), UB, 0, s>>>(A.rowptr, A.col, T.rowptr, T.col, tsrc,
                                                     A.nrows, nullptr, M.rowptr, M.col, ia, ib);
}

void symmetrize_numeric(const double* aval, const int32_t* ia, const int32_t* ib, Csr& M,
                        hipStream_t s) {
  if (M.nnz) k_sym_vals<<<nblocks(M.nnz, 256), 256, 0, s>>>(aval, ia, ib, M.val, M.nnz);
}


}  // namespace emin
