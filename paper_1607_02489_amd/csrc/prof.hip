// HIP-event profiler of kernel classes (see prof.h).
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include "chunk_cache.h"
#include "prof.h"

#include <map>
#include <mutex>
#include <set>

namespace emin {
namespace prof {
namespace {

struct Rec {
  int kind;
  double bytes, flops;
  hipEvent_t e0, e1;
};

std::mutex mu;
uint32_t kinds = 0;   // bit k: time kind k
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_OK(hipEventCreate(&e));
  return e;
}

}  // namespace

bool enabled(int kind) { return (kinds >> kind) & 1u; }

int begin(hipStream_t s, int kind, double bytes, double flops) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
  std::lock_guard<std::mutex> g(mu);
  Rec r{kind, bytes, flops, get_event(), get_event()};
  HIP_OK(hipEventRecord(r.e0, s));
  recs.push_back(r);
  return (int)recs.size() - 1;
}

bool begin_launch(hipStream_t s, int kind, double bytes, double flops, hipEvent_t* e0,
                  hipEvent_t* e1) {
  if (!enabled(kind)) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  std::lock_guard<std::mutex> g(mu);
  Rec r{kind, bytes, flops, get_event(), get_event()};
  recs.push_back(r);
  *e0 = r.e0;
  *e1 = r.e1;
  return true;
}

void end(int token, hipStream_t s) {
  std::lock_guard<std::mutex> g(mu);
  if (token >= 0 && token < (int)recs.size()) (void)hipEventRecord(recs[token].e1, s);
}

}  // namespace prof
}  // namespace emin

namespace emin {
namespace {
// the device side of the chunk cache: hipMalloc/hipFree, events as tokens
struct HipChunks {
  using Token = WorkToken;
  void* alloc(size_t bytes) {
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void free(void* p) { (void)hipFree(p); }
  // (hipErrorNotReady is an answer here, not an error: it is taken out of the
  // thread's last-error state, which a later launch check reads; with an
  // error already pending there the query is skipped, keeping that error)
  bool done(const Token& t) {
    if (!t) return true;
    if (hipPeekAtLastError() != hipSuccess) return false;
    const hipError_t q = hipEventQuery(t->e);
    if (q != hipSuccess) (void)hipGetLastError();
    return q == hipSuccess;
  }
  void wait(const Token& t) {
    if (t) (void)hipEventSynchronize(t->e);
  }
  [[noreturn]] void fail(const char* msg) {
    std::fprintf(stderr, "emin: %s\n", msg);
    std::abort();
  }
};
ChunkCache<HipChunks>& chunk_cache() {
  static ChunkCache<HipChunks>* c = new ChunkCache<HipChunks>();   // outlives exit-time releases
  return *c;
}
int current_device() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  return dev;
}
}  // namespace

void allow_lds(const void* f) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  if (done.count({f, dev})) return;
  int mx = 0;
  HIP_OK(hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  hipFuncAttributes fa;
  HIP_OK(hipFuncGetAttributes(&fa, f));
  HIP_OK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                             mx - (int)fa.sharedSizeBytes));
  done.insert({f, dev});
}

void* chunk_get(size_t bytes) { return chunk_cache().get(bytes, current_device()); }

void chunk_put(void* p, size_t bytes, WorkToken done) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  chunk_cache().put(p, bytes, dev, std::move(done));
}

// ---------------------------------------------------------------------------
// small read-backs through pinned, device-mapped host memory
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kSlotBytes = 4096;   // payload bytes per read-back
struct MappedSlot {
  unsigned char* h = nullptr;   // host address: [0, 64) sequence word, then payload
  unsigned char* d = nullptr;   // the same memory as the device sees it
  uint64_t seq = 0;
};

MappedSlot& mapped_slot() {
  thread_local MappedSlot per_dev[64];
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(EMIN_ERR_DEVICE, "device index");
  MappedSlot& m = per_dev[dev];
  if (!m.h) {
    void* h = nullptr;
    HIP_OK(hipHostMalloc(&h, 64 + kSlotBytes, hipHostMallocMapped | hipHostMallocCoherent));
    void* d = nullptr;
    HIP_OK(hipHostGetDevicePointer(&d, h, 0));
    *reinterpret_cast<volatile uint64_t*>(h) = 0;
    m.h = static_cast<unsigned char*>(h);
    m.d = static_cast<unsigned char*>(d);
  }
  return m;
}

// copies the payload into host memory, then (after a system-scope fence)
// the sequence number that tells the host the payload has arrived
__global__ void k_read_back(const unsigned char* src, int64_t n, unsigned char* slot,
                            uint64_t seq) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) slot[64 + i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    __hip_atomic_store(reinterpret_cast<uint64_t*>(slot), seq, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}
}  // namespace

void read_back(void* host, const void* dev, size_t bytes, hipStream_t s) {
  if (bytes > kSlotBytes) {
    HIP_OK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return;
  }
  MappedSlot& m = mapped_slot();
  const uint64_t seq = ++m.seq;
  k_read_back<<<1, 256, 0, s>>>(static_cast<const unsigned char*>(dev), (int64_t)bytes, m.d, seq);
  HIP_OK(hipGetLastError());
  // poll briefly (the common case: the stream is nearly drained); then wait
  // on the stream, which also reports a failed kernel
  const auto t0 = std::chrono::steady_clock::now();
  const volatile uint64_t* flag = reinterpret_cast<const volatile uint64_t*>(m.h);
  int n = 0;
  while (*flag != seq) {
    if ((++n & 255) == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(200)) {
      HIP_OK(hipStreamSynchronize(s));
      if (*flag != seq) throw Error(EMIN_ERR_DEVICE, "read-back did not arrive");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  std::memcpy(host, m.h + 64, bytes);
}
}  // namespace emin

extern "C" {

int64_t emin_release_cached(void) { return (int64_t)emin::chunk_cache().release_all(); }

emin_status emin_profile_enable(int enable) {
  std::lock_guard<std::mutex> g(emin::prof::mu);
  if (enable == 0) emin::prof::kinds = 0u;
  else if (enable & EMIN_PROF_ONLY) emin::prof::kinds = (uint32_t)enable & ((1u << EMIN_PROF_N) - 1u);
  else emin::prof::kinds = (1u << EMIN_PROF_N) - 1u;
  return EMIN_OK;
}

emin_status emin_profile_launches(emin_klaunch_t* out, int32_t cap, int32_t* n) {
  if (!n || cap < 0 || (cap && !out)) return EMIN_ERR_ARG;
  using namespace emin::prof;
  std::lock_guard<std::mutex> g(mu);
  int32_t k = 0;
  for (Rec& r : recs) {
    if (hipEventSynchronize(r.e1) != hipSuccess) return EMIN_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return EMIN_ERR_DEVICE;
    if (k < cap) out[k] = emin_klaunch_t{r.kind, 0, (double)ms, r.bytes, r.flops};
    k++;
    pool.push_back(r.e0);
    pool.push_back(r.e1);
  }
  recs.clear();
  *n = k;
  return EMIN_OK;
}

emin_status emin_profile_collect(emin_kstat_t* out, int32_t nkinds) {
  if (!out || nkinds <= 0) return EMIN_ERR_ARG;
  using namespace emin::prof;
  std::lock_guard<std::mutex> g(mu);
  for (int k = 0; k < nkinds; k++) out[k] = emin_kstat_t{0, 0.0, 0.0, 0.0};
  for (Rec& r : recs) {
    if (hipEventSynchronize(r.e1) != hipSuccess) return EMIN_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return EMIN_ERR_DEVICE;
    if (r.kind >= 0 && r.kind < nkinds) {
      out[r.kind].launches += 1;
      out[r.kind].total_ms += ms;
      out[r.kind].bytes += r.bytes;
      out[r.kind].flops += r.flops;
    }
    pool.push_back(r.e0);
    pool.push_back(r.e1);
  }
  recs.clear();
  return EMIN_OK;
}

}  // extern "C"
