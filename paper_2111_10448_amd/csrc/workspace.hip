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
#include "internal.h"

namespace pstt2 {

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
  for (void* p : a->spill) (void)hipFreeAsync(p, s);
  a->spill.clear();
  if (a->need > a->cap) {
    if (a->base) (void)hipFreeAsync(a->base, s);
    a->base = nullptr;
    a->cap = 0;
    const size_t want = round_up(a->need + a->need / 4);
    hipError_t e = hipMallocAsync((void**)&a->base, want, s);
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
  for (void* p : a->spill) (void)hipFreeAsync(p, s);
  a->spill.clear();
  if (a->base) (void)hipFreeAsync(a->base, s);
  a->base = nullptr;
  a->cap = a->off = a->need = 0;
}

hipError_t ws_alloc(void** p, size_t bytes, hipStream_t s) {
  Arena* a = current_arena();
  if (!a) return hipMallocAsync(p, bytes, s);
  const size_t b = round_up(bytes > 0 ? bytes : 1);
  a->need += b;
  if (a->off + b <= a->cap) {
    *p = a->base + a->off;
    a->off += b;
    return hipSuccess;
  }
  hipError_t e = hipMallocAsync(p, b, s);
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
  (void)hipFreeAsync(p, s);
}

}  // namespace pstt2
