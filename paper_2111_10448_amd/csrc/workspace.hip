// Device workspace for the library's internal temporaries.
//
// Outside an arena scope ws_alloc / ws_free are the stream-ordered allocator.
// Inside one (pstt2_recover binds the context's arena, tt_error a per-thread
// arena) they bump-allocate from one persistent buffer: the host cost of a
// temporary drops from a pool call (tens of microseconds around a stream
// synchronisation) to an add.  Requests that do not fit are served by the
// stream-ordered allocator and remembered; the next arena_begin releases them
// and regrows the buffer to the size the last pass needed, so from the second
// pass on every request fits.
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <unordered_map>

#include "internal.h"

namespace pstt2 {

// ---- device-memory accounting ----
// Every device allocation of the library goes through dev_malloc /
// dev_malloc_async and is released through dev_free / dev_free_async, which
// keep the live and peak byte counts and enforce the budget (PSTT2_MAX_BYTES
// in the environment, or pstt2_set_memory_limit).
namespace {
struct MemBook {
  std::mutex mu;
  std::unordered_map<void*, size_t> live;
  int64_t bytes = 0, peak = 0, limit = -1;
  MemBook() {
    if (const char* v = std::getenv("PSTT2_MAX_BYTES")) {
      char* end = nullptr;
      const long long b = std::strtoll(v, &end, 10);
      if (end != v && b > 0) limit = b;
    }
  }
};
MemBook& book() {
  static MemBook* b = new MemBook();   // never destroyed: frees may run during exit
  return *b;
}
bool book_reserve(size_t bytes) {
  MemBook& b = book();
  std::lock_guard<std::mutex> g(b.mu);
  if (b.limit > 0 && b.bytes + (int64_t)bytes > b.limit) return false;
  b.bytes += (int64_t)bytes;
  return true;
}
void book_commit(void* p, size_t bytes) {
  MemBook& b = book();
  std::lock_guard<std::mutex> g(b.mu);
  b.live[p] = bytes;
  b.peak = std::max(b.peak, b.bytes);
}
void book_cancel(size_t bytes) {
  MemBook& b = book();
  std::lock_guard<std::mutex> g(b.mu);
  b.bytes -= (int64_t)bytes;
}
void book_release(void* p) {
  MemBook& b = book();
  std::lock_guard<std::mutex> g(b.mu);
  auto it = b.live.find(p);
  if (it == b.live.end()) return;
  b.bytes -= (int64_t)it->second;
  b.live.erase(it);
}
std::atomic<int64_t> g_fault_after{-1};
}  // namespace

hipError_t dev_malloc_raw(void** p, size_t bytes) {
  *p = nullptr;
  if (!book_reserve(bytes)) return hipErrorOutOfMemory;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    book_cancel(bytes);
    return e;
  }
  book_commit(*p, bytes);
  return e;
}

hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (!book_reserve(bytes)) return hipErrorOutOfMemory;
  const hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    *p = nullptr;
    book_cancel(bytes);
    return e;
  }
  book_commit(*p, bytes);
  return e;
}

void dev_free(void* p) {
  if (!p) return;
  book_release(p);
  (void)hipFree(p);
}

void dev_free_async(void* p, hipStream_t s) {
  if (!p) return;
  book_release(p);
  (void)hipFreeAsync(p, s);
}

void mem_limit_set(int64_t bytes) {
  MemBook& b = book();
  std::lock_guard<std::mutex> g(b.mu);
  b.limit = bytes > 0 ? bytes : -1;
}

void mem_stats(int64_t* live, int64_t* peak, int64_t* limit) {
  MemBook& b = book();
  std::lock_guard<std::mutex> g(b.mu);
  if (live) *live = b.bytes;
  if (peak) *peak = b.peak;
  if (limit) *limit = b.limit;
}

void fault_arm(int64_t count) { g_fault_after.store(count < 0 ? -1 : count); }

bool fault_take() {
  int64_t v = g_fault_after.load();
  while (v >= 0) {
    if (g_fault_after.compare_exchange_weak(v, v - 1)) return v == 0;
  }
  return false;
}

namespace {
constexpr size_t kAlign = 256;
size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
}  // namespace

Arena*& current_arena() {
  thread_local Arena* a = nullptr;
  return a;
}

ArenaScope::ArenaScope(Arena* a) : prev(current_arena()) { current_arena() = a; }
ArenaScope::~ArenaScope() { current_arena() = prev; }

hipError_t arena_begin(Arena* a, hipStream_t s) {
  for (void* p : a->spill) dev_free_async(p, s);
  a->spill.clear();
  if (a->need > a->cap) {
    if (a->base) dev_free_async(a->base, s);
    a->base = nullptr;
    a->cap = 0;
    const size_t want = round_up(a->need + a->need / 4);
    hipError_t e = dev_malloc_async((void**)&a->base, want, s);
    if (e != hipSuccess) {
      a->base = nullptr;
      a->need = 0;
      return e;
    }
    a->cap = want;
  }
  a->off = 0;
  a->need = 0;
  return hipSuccess;
}

void arena_release(Arena* a, hipStream_t s) {
  for (void* p : a->spill) dev_free_async(p, s);
  a->spill.clear();
  if (a->base) dev_free_async(a->base, s);
  a->base = nullptr;
  a->cap = a->off = a->need = 0;
}

hipError_t ws_alloc(void** p, size_t bytes, hipStream_t s) {
  Arena* a = current_arena();
  if (!a) return dev_malloc_async(p, bytes, s);
  const size_t b = round_up(bytes > 0 ? bytes : 1);
  a->need += b;
  if (a->off + b <= a->cap) {
    *p = a->base + a->off;
    a->off += b;
    return hipSuccess;
  }
  hipError_t e = dev_malloc_async(p, b, s);
  if (e == hipSuccess) a->spill.push_back(*p);
  return e;
}

void ws_free(void* p, hipStream_t s) {
  if (!p) return;
  Arena* a = current_arena();
  if (a) {
    const char* c = (const char*)p;
    if (c >= a->base && c < a->base + a->cap) return;
    for (void* q : a->spill)
      if (q == p) return;   // released by the next arena_begin
  }
  dev_free_async(p, s);
}

}  // namespace pstt2
