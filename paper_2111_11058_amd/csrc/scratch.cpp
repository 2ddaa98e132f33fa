// Cache of device scratch blocks.
//
// On this runtime the stream-ordered allocator (hipMallocAsync /
// hipFreeAsync) costs from about a hundred microseconds to a few
// milliseconds per call, whatever the size and the pool's release threshold,
// and multi-gigabyte blocks far more; with some ninety scratch blocks per
// CBF build, projection and solve, that host time left the device idle for
// a sixth of a small problem's step.  Every scratch block therefore comes
// from plain device allocations that are kept after use and handed out
// again:
//  * blocks below kBigScratch are rounded up to a power of two and reused
//    for requests of the same class; larger ones are reused for requests of
//    at least half their size;
//  * a released block carries an event recorded on the releasing stream, and
//    the next user's stream waits on it, so reuse is ordered after every
//    operation queued before the release, on any stream;
//  * before a stream is destroyed, its owner synchronises it and calls
//    scratch_forget_stream: the blocks it released are then complete, their
//    events are destroyed and they are tagged with no stream, so the cache
//    never waits on, synchronises or compares the handle or an event of a
//    destroyed stream (a new stream may reuse the handle value);
//  * among the cached blocks that fit, one released on the requesting stream
//    is taken first (stream order already puts it after its last use), then
//    one released on another stream.  A block released on a library side
//    stream is taken by another stream only if a new allocation fails, so
//    that the CMP inverse formed there does not hold back the caller's
//    projection through the cache.  (Choices go by the releasing stream
//    alone; the cache queries no event.)  A block whose stream was
//    forgotten counts as released on the requesting stream;
//  * the bytes cached per device are capped at kCacheCap (the oldest blocks
//    are freed first), and if an allocation fails, the device's cached blocks
//    are freed (after their events complete) and the allocation is retried.
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

namespace cbfm {

namespace {

constexpr size_t kCacheCap = (size_t)64 << 30;
constexpr size_t kMinBlock = 512;

size_t block_size(size_t bytes) {
  if (bytes >= kBigScratch) return bytes;
  size_t b = kMinBlock;
  while (b < bytes) b <<= 1;
  return b;
}

struct Block {
  void* p;
  size_t bytes;
  int dev;
  hipEvent_t ready;    // recorded at the release; nullptr: known complete
  hipStream_t stream;  // the releasing stream; nullptr once forgotten
  bool forgotten;      // the releasing stream was destroyed (see scratch_forget_stream)
};

struct Cache {
  std::mutex mu;
  std::vector<hipStream_t> side;                   // library side streams
  std::vector<Block> free;                         // in release order
  std::vector<std::pair<int, hipEvent_t>> events;  // spare events and their devices
};

// never destroyed: the runtime may be torn down before static destructors run
Cache& cache() {
  static Cache* c = new Cache;
  return *c;
}

hipEvent_t take_event(int dev) {
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& ev = cache().events;
    for (size_t i = ev.size(); i-- > 0;)
      if (ev[i].first == dev) {
        const hipEvent_t e = ev[i].second;
        ev[i] = ev.back();
        ev.pop_back();
        return e;
      }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// (call with the cache lock held)
void spare_event(int dev, hipEvent_t e) { cache().events.push_back({dev, e}); }

void free_blocks(std::vector<Block>& drop) {
  for (Block& b : drop) {
    if (b.ready) (void)hipEventSynchronize(b.ready);
    (void)hipFree(b.p);
    device_bytes_add(-(int64_t)b.bytes);
    if (b.ready) {
      std::lock_guard<std::mutex> lk(cache().mu);
      spare_event(b.dev, b.ready);
    }
  }
  drop.clear();
}

void trim(int dev) {
  std::vector<Block> drop;
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    for (size_t i = 0; i < f.size();) {
      if (f[i].dev == dev) {
        drop.push_back(f[i]);
        f.erase(f.begin() + (ptrdiff_t)i);
      } else {
        ++i;
      }
    }
  }
  free_blocks(drop);
}

}  // namespace

void* scratch_alloc(size_t bytes, hipStream_t s, size_t* block) {
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  const size_t want = block_size(bytes);
  const bool big = want >= kBigScratch;
  auto fits = [&](const Block& b) {
    return b.dev == dev && (big ? b.bytes >= want && b.bytes <= 2 * want : b.bytes == want);
  };
  // take cached block i (lock held on entry, released on return)
  auto take = [&](std::unique_lock<std::mutex>& lk, size_t i) {
    const Block b = cache().free[i];
    *block = b.bytes;
    cache().free.erase(cache().free.begin() + (ptrdiff_t)i);  // (keeps the release order)
    lk.unlock();
    if (b.ready) {
      if (hipStreamWaitEvent(s, b.ready, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventSynchronize(b.ready);  // keep the ordering before handing the block out
      }
    }
    lk.lock();
    if (b.ready) spare_event(dev, b.ready);  // re-recording later leaves a queued wait as it was
    return b.p;
  };
  size_t busy = SIZE_MAX;  // a fitting block released on a side stream
  {
    std::unique_lock<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    const auto& side = cache().side;
    size_t same = SIZE_MAX, other = SIZE_MAX;
    for (size_t i = 0; i < f.size(); ++i) {
      if (!fits(f[i])) continue;
      size_t& slot = f[i].forgotten || f[i].stream == s ? same
                     : std::find(side.begin(), side.end(), f[i].stream) != side.end() ? busy
                                                                                         : other;
      if (slot == SIZE_MAX || f[i].bytes < f[slot].bytes) slot = i;
    }
    if (same != SIZE_MAX) return take(lk, same);
    if (other != SIZE_MAX) return take(lk, other);
  }
  void* p = nullptr;
  *block = want;
  if (hipMalloc(&p, want) == hipSuccess) {
    device_bytes_add((int64_t)want);
    return p;
  }
  (void)hipGetLastError();
  if (busy != SIZE_MAX) {  // wait for a block in use rather than fail
    std::unique_lock<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    for (size_t i = 0; i < f.size(); ++i)
      if (fits(f[i])) return take(lk, i);
  }
  trim(dev);
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{CBFM_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
  }
  device_bytes_add((int64_t)want);
  return p;
}

void scratch_release(void* p, size_t block, hipStream_t s) {
  int dev = 0;
  hipEvent_t ev = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || (ev = take_event(dev)) == nullptr || hipEventRecord(ev, s) != hipSuccess) {
    // no way to order a later reuse: wait for the stream, then free
    (void)hipGetLastError();
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    device_bytes_add(-(int64_t)block);
    return;
  }
  std::vector<Block> drop;
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    f.push_back({p, block, dev, ev, s, false});
    size_t held = 0;
    for (const Block& b : f)
      if (b.dev == dev) held += b.bytes;
    // oldest first: entries are appended in release order
    for (size_t i = 0; held > kCacheCap && i < f.size();) {
      if (f[i].dev == dev) {
        held -= f[i].bytes;
        drop.push_back(f[i]);
        f.erase(f.begin() + (ptrdiff_t)i);
      } else {
        ++i;
      }
    }
  }
  free_blocks(drop);
}

void scratch_forget_stream(hipStream_t s) {
  std::vector<hipEvent_t> done;
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    for (Block& b : cache().free)
      if (!b.forgotten && b.stream == s) {
        if (b.ready) done.push_back(b.ready);
        b.ready = nullptr;
        b.stream = nullptr;
        b.forgotten = true;
      }
  }
  // the caller synchronised s: these events are complete and never used again
  for (hipEvent_t e : done) (void)hipEventDestroy(e);
}

void scratch_trim_to(size_t limit) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::vector<Block> drop;
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    size_t held = 0;
    for (const Block& b : f)
      if (b.dev == dev) held += b.bytes;
    for (size_t i = 0; held > limit && i < f.size();) {
      if (f[i].dev == dev) {
        held -= f[i].bytes;
        drop.push_back(f[i]);
        f.erase(f.begin() + (ptrdiff_t)i);
      } else {
        ++i;
      }
    }
  }
  free_blocks(drop);
}

void scratch_side_stream(hipStream_t s) {
  std::lock_guard<std::mutex> lk(cache().mu);
  cache().side.push_back(s);
}

size_t scratch_cached_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> lk(cache().mu);
  size_t held = 0;
  for (const Block& b : cache().free)
    if (b.dev == dev) held += b.bytes;
  return held;
}

}  // namespace cbfm

// ------------------------------------------------------------ allocator hook
namespace cbfm {
namespace {
std::mutex g_hook_mu;
cbfm_alloc_fn g_alloc = nullptr;
cbfm_release_fn g_release = nullptr;
std::mutex g_bytes_mu;
int64_t g_bytes = 0, g_peak = 0;
}  // namespace

void device_bytes_add(int64_t delta) {
  std::lock_guard<std::mutex> lk(g_bytes_mu);
  g_bytes += delta;
  g_peak = std::max(g_peak, g_bytes);
}

void* hooked_alloc(size_t bytes, hipStream_t s, ReleaseFn* release) {
  cbfm_alloc_fn a;
  {
    std::lock_guard<std::mutex> lk(g_hook_mu);
    a = g_alloc;
    *release = g_release;
  }
  if (!a) return nullptr;
  return a(bytes, static_cast<void*>(s));
}
}  // namespace cbfm

using namespace cbfm;

extern "C" cbfm_status cbfm_set_allocator(cbfm_alloc_fn alloc, cbfm_release_fn release) {
  return guarded([&] {
    CBFM_REQUIRE((alloc == nullptr) == (release == nullptr), CBFM_E_ARG, "set both routines or neither");
    {
      std::lock_guard<std::mutex> lk(g_hook_mu);
      g_alloc = alloc;
      g_release = release;
    }
    // blocks cached from hipMalloc are no longer handed out: free them
    if (alloc) scratch_trim_to(0);
  });
}

extern "C" cbfm_status cbfm_memory_stats(int64_t* held, int64_t* peak, int64_t* cached) {
  return guarded([&] {
    {
      std::lock_guard<std::mutex> lk(g_bytes_mu);
      if (held) *held = g_bytes;
      if (peak) *peak = g_peak;
    }
    if (cached) *cached = (int64_t)scratch_cached_bytes();
  });
}
