// Process-wide cache of device memory chunks, with an ownership ledger.
//
// Handles return their chunks here instead of freeing them (a free waits for
// the whole device), and new allocations take cached chunks first.  Host
// threads share the cache, so two rules keep a chunk from being handed to
// one owner while another's work may still touch it:
//   - every chunk is either leased (to exactly one owner) or cached; the
//     ledger checks each transition, so a chunk handed out twice or given
//     back twice stops the process with a message instead of corrupting
//     another owner's data;
//   - a chunk is given back with a completion token (an event recorded on the
//     stream that last queued work on it); it is handed out again only once
//     that token reports completion, else a fresh chunk is allocated.
// Chunks of one device are never handed to another.
//
// Host code only: the device side (allocation, events) comes from Backend,
// so the same logic runs under a host-only test backend.  Backend provides
//   Token                      copyable; Token{} means "nothing queued"
//   void* alloc(size_t)        nullptr on failure
//   void free(void*)
//   bool done(const Token&)    the queued work has completed
//   void wait(const Token&)    blocks until it has
//   void fail(const char*)     a ledger violation (does not return)
#pragma once
#include <cstddef>
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

namespace emin {

template <class Backend>
class ChunkCache {
 public:
  using Token = typename Backend::Token;
  explicit ChunkCache(Backend be = Backend()) : be_(std::move(be)) {}

  // a chunk of exactly `bytes` on device `dev`, leased to the caller
  void* get(size_t bytes, int dev) {
    {
      std::lock_guard<std::mutex> g(mu_);
      auto range = cache_.equal_range(Key{dev, bytes});
      for (auto it = range.first; it != range.second; ++it) {
        if (!be_.done(it->second.tok)) continue;
        void* p = it->second.p;
        cache_.erase(it);
        Entry& e = ledger_at(p);
        if (e.leased) be_.fail("chunk cache: a cached chunk is also leased");
        if (e.bytes != bytes || e.dev != dev) be_.fail("chunk cache: ledger size or device differs");
        e.leased = true;
        return p;
      }
    }
    void* p = be_.alloc(bytes);
    if (!p) return nullptr;
    std::lock_guard<std::mutex> g(mu_);
    auto it = ledger_.find(p);
    if (it != ledger_.end()) be_.fail("chunk cache: a fresh allocation is already in the ledger");
    ledger_.emplace(p, Entry{bytes, dev, true});
    return p;
  }

  // gives back a leased chunk; tok completes when the last work queued on it
  // has (Token{} when none is queued)
  void put(void* p, size_t bytes, int dev, Token tok) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = ledger_.find(p);
    if (it == ledger_.end()) be_.fail("chunk cache: a chunk given back was never handed out");
    Entry& e = it->second;
    if (!e.leased) be_.fail("chunk cache: a chunk given back twice");
    if (e.bytes != bytes || e.dev != dev) be_.fail("chunk cache: a chunk given back with another size or device");
    e.leased = false;
    cache_.emplace(Key{dev, bytes}, Cached{p, std::move(tok)});
  }

  // frees every cached chunk (waiting for its queued work); returns the bytes
  size_t release_all() {
    std::lock_guard<std::mutex> g(mu_);
    size_t freed = 0;
    for (auto& kv : cache_) {
      be_.wait(kv.second.tok);
      be_.free(kv.second.p);
      ledger_.erase(kv.second.p);
      freed += kv.first.second;
    }
    cache_.clear();
    return freed;
  }

  size_t leased() const {
    std::lock_guard<std::mutex> g(mu_);
    size_t n = 0;
    for (const auto& kv : ledger_) n += kv.second.leased ? 1 : 0;
    return n;
  }
  size_t cached() const {
    std::lock_guard<std::mutex> g(mu_);
    return cache_.size();
  }
  Backend& backend() { return be_; }

 private:
  using Key = std::pair<int, size_t>;   // device, bytes
  struct Cached {
    void* p;
    Token tok;
  };
  struct Entry {
    size_t bytes;
    int dev;
    bool leased;
  };
  Entry& ledger_at(void* p) {
    auto it = ledger_.find(p);
    if (it == ledger_.end()) be_.fail("chunk cache: a cached chunk is missing from the ledger");
    return it->second;
  }
  Backend be_;
  mutable std::mutex mu_;
  std::multimap<Key, Cached> cache_;
  std::unordered_map<void*, Entry> ledger_;
};

}  // namespace emin
