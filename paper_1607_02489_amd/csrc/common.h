// Shared device/host infrastructure of the EMIN-AMG HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/emin.h"

namespace emin {

// ---------------------------------------------------------------------------
// errors: host code throws, the C-ABI layer converts to emin_status
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  emin_status code;
  Error(emin_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess)                                                      \
      throw ::emin::Error(EMIN_ERR_DEVICE, std::string(#x) + ": " +            \
                                               hipGetErrorString(e_));         \
  } while (0)

// device-side error flags (bit per kind), read back by host syncs
enum DevErr : int {
  DERR_CAPACITY = 1,   // a fixed-capacity per-row buffer overflowed
  DERR_PATTERN = 2,    // malformed CSR (unsorted / duplicate / out of range)
  DERR_VALUE = 4,      // NaN / Inf input
  DERR_COLOCATE = 8,   // a coarse pressure without a co-located coarse velocity
};

// ---------------------------------------------------------------------------
// device memory owned by a handle
// ---------------------------------------------------------------------------
// The completion point of queued work: an event, destroyed with its last
// owner.  An empty token stands for "no work queued".
struct EventBox {
  hipEvent_t e = nullptr;
  EventBox() = default;
  EventBox(const EventBox&) = delete;
  EventBox& operator=(const EventBox&) = delete;
  ~EventBox() {
    if (e) (void)hipEventDestroy(e);
  }
};
using WorkToken = std::shared_ptr<EventBox>;

// Process-wide cache of device chunks (with an ownership ledger): handles
// return their chunks here instead of calling hipFree (which would wait for
// the whole device), and new allocations on the same device take cached
// chunks first, once the work last queued on them has completed.
// emin_release_cached() frees the cache.
void* chunk_get(size_t bytes);
void chunk_put(void* p, size_t bytes, WorkToken done);

// Lets kernel f take up to the device's LDS per block (less its static LDS)
// as dynamic LDS.  Set once per kernel and device, under a lock, so host
// threads launching f with different sizes never race on the limit.
void allow_lds(const void* f);

class Arena {
 public:
  Arena() = default;
  // a fixed buffer instead of chunks: allocation only bumps within
  // [base, base + cap) and throws EMIN_ERR_CAPACITY beyond it (no device
  // allocation ever happens)
  Arena(void* base, size_t cap) : fixed_(true), cur_(static_cast<char*>(base)), left_(cap) {}
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena() { release(); }
  // chunks from a caller's allocator instead of the library's cache (set
  // before the first allocation)
  void use_allocator(const emin_allocator_t& a) {
    if (!chunks_.empty() || fixed_) throw Error(EMIN_ERR_ARG, "allocator set after allocation");
    if (!a.alloc || !a.free) throw Error(EMIN_ERR_ARG, "allocator without alloc or free");
    al_ = a;
    has_al_ = true;
  }
  // bump allocation from 64 MiB chunks (few allocations per handle)
  template <class T>
  T* alloc(size_t n) {
    size_t b = (n ? n : 1) * sizeof(T);
    b = (b + 255) & ~size_t(255);
    if (b > left_ && fixed_) throw Error(EMIN_ERR_CAPACITY, "scratch buffer capacity exceeded");
    if (b > left_) {
      const size_t chunk = b > kChunk ? b : kChunk;
      void* p = has_al_ ? al_.alloc(chunk, al_.ctx) : chunk_get(chunk);
      if (!p) throw Error(EMIN_ERR_OOM, "device allocation failed");
      if (has_al_ && (reinterpret_cast<uintptr_t>(p) & 255)) {
        al_.free(p, al_.ctx);
        throw Error(EMIN_ERR_ARG, "allocator returned memory not 256-byte aligned");
      }
      chunks_.push_back({p, chunk});
      bytes_ += chunk;
      cur_ = static_cast<char*>(p);
      left_ = chunk;
    }
    void* r = cur_;
    cur_ += b;
    left_ -= b;
    return static_cast<T*>(r);
  }
  // Notes that work using this arena's memory has been queued on s up to
  // now (the arena keeps the latest such point, made to follow the previous
  // one when the stream differs).  Not while s is being captured into a
  // graph: the replays of a graph are the caller's to finish before the
  // release.  On any failure it waits for s instead.
  void used_on(hipStream_t s) noexcept {
    if (fixed_ || chunks_.empty()) return;
    // errors of the calls below are handled here (by waiting instead): a
    // clean last-error state is left clean for the caller's launch checks
    struct KeepClean {
      bool clean = hipPeekAtLastError() == hipSuccess;
      ~KeepClean() {
        if (clean) (void)hipGetLastError();
      }
    } keep;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
      (void)hipStreamSynchronize(s);
      return;
    }
    if (cs != hipStreamCaptureStatusNone) return;
    if (last_ && last_s_ != s && hipStreamWaitEvent(s, last_->e, 0) != hipSuccess)
      (void)hipEventSynchronize(last_->e);
    if (!last_) {
      try {
        last_ = std::make_shared<EventBox>();
      } catch (...) {
        (void)hipStreamSynchronize(s);
        return;
      }
      if (hipEventCreateWithFlags(&last_->e, hipEventDisableTiming) != hipSuccess) {
        last_->e = nullptr;
        last_.reset();
        (void)hipStreamSynchronize(s);
        return;
      }
    }
    if (hipEventRecord(last_->e, s) != hipSuccess) (void)hipStreamSynchronize(s);
    last_s_ = s;
  }
  // Gives the chunks back.  Work queued on them and noted by used_on() may
  // still be running: the cache hands them out again only after it has
  // completed.  A caller's allocator gets them back after it has completed.
  void release() {
    if (fixed_) return;
    for (auto& c : chunks_) {
      if (has_al_) {
        if (last_) (void)hipEventSynchronize(last_->e);
        al_.free(c.first, al_.ctx);
      } else {
        chunk_put(c.first, c.second, last_);
      }
    }
    chunks_.clear();
    last_.reset();
    last_s_ = nullptr;
    bytes_ = 0;
    cur_ = nullptr;
    left_ = 0;
  }
  size_t bytes() const { return bytes_; }

 private:
  static constexpr size_t kChunk = size_t(64) << 20;
  bool fixed_ = false;
  bool has_al_ = false;
  emin_allocator_t al_{};
  std::vector<std::pair<void*, size_t>> chunks_;
  WorkToken last_;                 // latest point of queued work (used_on)
  hipStream_t last_s_ = nullptr;   // the stream it was recorded on
  size_t bytes_ = 0;
  char* cur_ = nullptr;
  size_t left_ = 0;
};

// Notes, on leaving its scope (normally or by an exception), that work
// using the arena's memory was queued on s (Arena::used_on).
class StreamUse {
 public:
  StreamUse(Arena& a, hipStream_t s) : a_(a), s_(s) {}
  StreamUse(const StreamUse&) = delete;
  StreamUse& operator=(const StreamUse&) = delete;
  ~StreamUse() { a_.used_on(s_); }

 private:
  Arena& a_;
  hipStream_t s_;
};

// a CSR matrix in device memory (rowptr int64, col int32, val double/float)
struct Csr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int64_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};

struct CsrView {  // read-only borrowed input
  int64_t nrows = 0, ncols = 0, nnz = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
};

inline CsrView view(const Csr& a) { return {a.nrows, a.ncols, a.nnz, a.rowptr, a.col, a.val}; }

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Copies bytes (device) to host once the work queued on s before this call
// has completed.  Small read-backs go through pinned, device-mapped host
// memory of the calling thread: a one-block kernel writes them there and the
// host polls for their arrival (a few microseconds, against tens for a copy
// to pageable memory and a stream synchronisation).
void read_back(void* host, const void* dev, size_t bytes, hipStream_t s);

template <class T>
inline T d2h(const T* p, hipStream_t s) {
  T v;
  read_back(&v, p, sizeof(T), s);
  return v;
}

// message of the last error raised on this thread (emin_last_error)
void set_last_error(const char* msg);

// zero a device buffer with a kernel (graph-capturable; bytes % 4 == 0)
void zero_bytes(void* p, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------------------
// sparse building blocks (sparse.hip)
// ---------------------------------------------------------------------------
// max |i - j| over the entries of a square pattern (a graph's index bandwidth)
int64_t index_bandwidth(const int64_t* rp, const int32_t* col, int64_t n, hipStream_t s,
                        Arena& ar);
// the same two maxima left in device memory (*out, no read-back)
void index_bandwidth_dev(const int64_t* rp, const int32_t* col, int64_t n,
                         unsigned long long* out, hipStream_t s);
void max_row_len_dev(const int64_t* rp, int64_t n, unsigned long long* out, hipStream_t s);
// longest row of a CSR (synchronises the stream)
int64_t max_row_len(const int64_t* rp, int64_t n, hipStream_t s, Arena& ar);
// largest value of a non-negative int32 array (synchronises the stream)
int64_t max_row_len_i32(const int32_t* a, int64_t n, hipStream_t s, Arena& ar);
// in-place inclusive scan of a[0..n)
void scan_inclusive(int64_t* a, int64_t n, hipStream_t s, Arena& ar);
// counts written to rowptr[1..n]; rowptr[0] = 0 set here; returns total
int64_t rowptr_from_counts(int64_t* rowptr, int64_t n, hipStream_t s, Arena& ar);

// transpose: builds the pattern of A^T and src[p] = entry of A feeding At[p]
// (rows of At in ascending original-row order)
void transpose_pattern(const CsrView& A, Csr& At, int32_t*& src, hipStream_t s, Arena& ar);
void gather_values(const double* in, const int32_t* src, double* out, int64_t n, hipStream_t s);

// C = A*B: symbolic (pattern) once, numeric any number of times.  For every
// (i,j), c_ij accumulates a_ik*b_kj over k in ascending order of A's row,
// each product and sum rounded separately (bit-reproducible); in a row of
// more than SPGEMM_SPLIT entries of A, over each chunk of SPGEMM_SPLIT
// entries so, then the chunk sums in chunk order.  The symbolic
// pass reads back once (twice when rows exceed the window bitmap); an overflow
// seen only by its fill pass is ORed into *derr (DERR_CAPACITY) for the caller
// to check, or thrown at once when derr is null.
struct SpgemmPlan {
  int64_t max_row = 0;  // longest output row
  int64_t max_words = 0;  // widest column span of an output row, in 32-bit words
  int g_num = 16;       // lanes per row in the numeric kernel
  // rows with more than SPGEMM_SPLIT entries of A (and at most SPGEMM_SPLIT_NC
  // outputs) are summed in chunks of SPGEMM_SPLIT entries, one work item per
  // chunk, then the chunk sums are added in chunk order
  int64_t ntasks = 0;               // (row, chunk) work items
  const int32_t* task_row = nullptr;
  const int32_t* task_chunk = nullptr;
  const int64_t* poff = nullptr;    // per row: offset of its chunk sums, -1 when not split
  double* part = nullptr;           // chunk sums (8 bytes per value; FP32 uses the low half)
  int64_t max_arow = 0;             // longest row of A
};
constexpr int SPGEMM_SPLIT = 512;
constexpr int SPGEMM_SPLIT_NC = 1024;
// Device memory for stream-ordered temporaries that a handle reuses (the
// stored bitmaps of the symbolic products): grown on demand, never shrunk,
// and released by the owner once its queued work has completed.
struct Scratch {
  Arena ar;
  void* p = nullptr;
  size_t cap = 0;
  void* get(size_t b) {
    if (b > cap) {
      p = ar.alloc<char>(b);
      cap = b;
    }
    return p;
  }
  void release() {
    ar.release();
    p = nullptr;
    cap = 0;
  }
};
// the stored bitmaps of one symbolic product are kept up to this size (else
// the product is formed once per pass)
constexpr size_t kStoredBitmapMax = size_t(2) << 30;
// split: rows of more than SPGEMM_SPLIT entries of A may be summed in chunks
// (only for products whose values need not equal the single ascending chain
// bit for bit).  scratch: keep each output row's window bitmap between the
// count and fill passes in it (one formation of the products instead of
// two); the caller keeps the scratch memory until the queued work is done.
void spgemm_symbolic(const CsrView& A, const CsrView& B, Csr& C, SpgemmPlan& plan,
                     hipStream_t s, Arena& ar, int* derr, bool split = false,
                     Scratch* scratch = nullptr);
void spgemm_numeric(const CsrView& A, const CsrView& B, const Csr& C, const SpgemmPlan& plan,
                    hipStream_t s);
// C = A A^T (B of the symbolic pass was A^T): when A has at most 256 rows,
// some longer than SPGEMM_SPLIT, c_ij as the dot product of rows i and j of A
// over their common columns in ascending order -- the same products summed in
// the same order as spgemm_numeric, so the same bits -- with one lane per
// output entry; otherwise spgemm_numeric
void spgemm_numeric_aat(const CsrView& A, const CsrView& At, const Csr& C, const SpgemmPlan& plan,
                        hipStream_t s);
// FP32 values and accumulation (mixed-precision RAP); result to cval32, or
// converted to FP64 into cval64 when that is non-null
void spgemm_numeric_f32(const CsrView& A, const float* aval, const CsrView& B, const float* bval,
                        const Csr& C, float* cval32, double* cval64, const SpgemmPlan& plan,
                        hipStream_t s);
void gather_values_f(const float* in, const int32_t* src, float* out, int64_t n, hipStream_t s);

// filter of eq. (e:filtering) with lumping; keep mask per entry of A; dir
// (optional): the rows' Dirichlet flags from the same pass (1 where no
// off-diagonal value of the row is nonzero)
void diag_of(const CsrView& A, double* d, hipStream_t s);
void filter_symbolic(const CsrView& A, double tau1, const double* d, uint8_t* keep, Csr& At,
                     hipStream_t s, Arena& ar, uint8_t* dir = nullptr);
void filter_numeric(const CsrView& A, const uint8_t* keep, const double* d, const Csr& At,
                    hipStream_t s);
// M = (A + A^T)/2 on the union pattern; ia/ib = entry of A / of A (transposed
// position) feeding each entry of M, -1 if absent
void symmetrize_symbolic(const Csr& A, Csr& M, int32_t*& ia, int32_t*& ib, hipStream_t s,
                         Arena& ar);
void symmetrize_numeric(const double* aval, const int32_t* ia, const int32_t* ib, Csr& M,
                        hipStream_t s);
void validate_csr(const CsrView& A, bool values, int* derr, hipStream_t s);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
// XCD-aware block order: the hardware deals consecutive blocks round-robin to
// the 8 XCDs; remapping gives every XCD one contiguous range of rows, so the
// neighbour rows a block gathers are likely already in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8, x = b % 8, j = b / 8;
  return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, 64);
}

// ballot restricted to the caller's aligned group of G lanes (bit t = lane t
// of the group); lanes outside the group do not count
template <int G>
__device__ __forceinline__ uint64_t group_ballot(bool p) {
  const uint64_t b = __ballot(p);
  if (G == 64) return b;
  const int base = (int)(threadIdx.x & 63) & ~(G - 1);
  return (b >> base) & ((1ull << G) - 1ull);
}

// lexicographic (key, index) minimum across a full 64-lane wave
// Wave-wide reductions on the DPP network (row shifts, then the two row
// broadcasts), which leave the result in lane 63; it is then read out as a
// wave-uniform value.  Every lane of the wave must be active.  Lanes whose
// DPP source lies outside the row (or whose row is masked off) keep the
// identity passed as "old".
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double ident, double v) {
  const unsigned long long o = (unsigned long long)__double_as_longlong(ident);
  const unsigned long long x = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)x, CTRL, ROWS, 0xF,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(x >> 32),
                                             CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double wave_min_f64(double v) {
  const double I = __builtin_inf();
  double t;
  t = dpp_f64<0x111, 0xF>(I, v); v = t < v ? t : v;   // row_shr:1
  t = dpp_f64<0x112, 0xF>(I, v); v = t < v ? t : v;   // row_shr:2
  t = dpp_f64<0x114, 0xF>(I, v); v = t < v ? t : v;   // row_shr:4
  t = dpp_f64<0x118, 0xF>(I, v); v = t < v ? t : v;   // row_shr:8
  t = dpp_f64<0x142, 0xA>(I, v); v = t < v ? t : v;   // row_bcast:15
  t = dpp_f64<0x143, 0xC>(I, v); v = t < v ? t : v;   // row_bcast:31
  const unsigned long long x = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
  const int I = INT32_MAX;
  int t;
  t = __builtin_amdgcn_update_dpp(I, v, 0x111, 0xF, 0xF, false); v = t < v ? t : v;
  t = __builtin_amdgcn_update_dpp(I, v, 0x112, 0xF, 0xF, false); v = t < v ? t : v;
  t = __builtin_amdgcn_update_dpp(I, v, 0x114, 0xF, 0xF, false); v = t < v ? t : v;
  t = __builtin_amdgcn_update_dpp(I, v, 0x118, 0xF, 0xF, false); v = t < v ? t : v;
  t = __builtin_amdgcn_update_dpp(I, v, 0x142, 0xA, 0xF, false); v = t < v ? t : v;
  t = __builtin_amdgcn_update_dpp(I, v, 0x143, 0xC, 0xF, false); v = t < v ? t : v;
  return __builtin_amdgcn_readlane(v, 63);
}

// lexicographic (key, index) minimum over the wave, wave-uniform result:
// the smallest key first, then the smallest index among the lanes holding it
__device__ __forceinline__ void wave_argmin(double& k, int32_t& i) {
  const double km = wave_min_f64(k);
  i = wave_min_i32(k == km ? i : INT32_MAX);
  k = km;
}

}  // namespace emin
