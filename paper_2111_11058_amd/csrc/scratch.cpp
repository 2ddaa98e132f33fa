// Cache of large device scratch blocks.
//
// Freeing and re-mapping multi-gigabyte stream-ordered allocations
// (hipMallocAsync / hipFreeAsync) costs tens to hundreds of milliseconds
// each on this runtime once the pool has been used, which dominated the
// panelled projection of large meshes (panels of tens of GB).  Blocks of at
// least kBigScratch bytes therefore come from plain device allocations that
// are kept after use and handed out again.  A released block carries an
// event recorded on the releasing stream; the next user's stream waits on
// it, so reuse is ordered after every operation queued before the release.
// If an allocation fails, the cached blocks of that device are freed (after
// their events complete) and the allocation is retried; the blocks cached
// per device are capped at kCacheCap bytes (the oldest are freed first).
#include <mutex>
#include <vector>

#include "internal.h"

namespace cbfm {

namespace {

constexpr size_t kCacheCap = (size_t)64 << 30;

struct Block {
  void* p;
  size_t bytes;
  int dev;
  hipEvent_t ready;
};

struct Cache {
  std::mutex mu;
  std::vector<Block> free;
};

// never destroyed: the runtime may be torn down before static destructors run
Cache& cache() {
  static Cache* c = new Cache;
  return *c;
}

void trim(int dev) {
  std::vector<Block> drop;
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    for (size_t i = 0; i < f.size();) {
      if (f[i].dev == dev) {
        drop.push_back(f[i]);
        f[i] = f.back();
        f.pop_back();
      } else {
        ++i;
      }
    }
  }
  for (Block& b : drop) {
    (void)hipEventSynchronize(b.ready);
    (void)hipEventDestroy(b.ready);
    (void)hipFree(b.p);
  }
}

}  // namespace

void* big_alloc(size_t bytes, hipStream_t s) {
  int dev = 0;
  CBFM_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    // the smallest cached block that fits and wastes at most half of itself
    size_t best = f.size();
    for (size_t i = 0; i < f.size(); ++i)
      if (f[i].dev == dev && f[i].bytes >= bytes && f[i].bytes <= 2 * bytes &&
          (best == f.size() || f[i].bytes < f[best].bytes))
        best = i;
    if (best < f.size()) {
      const Block b = f[best];
      f.erase(f.begin() + (ptrdiff_t)best);  // (keeps the release order)
      const hipError_t e = hipStreamWaitEvent(s, b.ready, 0);
      (void)hipEventDestroy(b.ready);
      if (e != hipSuccess) {
        (void)hipDeviceSynchronize();  // keep the ordering before handing the block out
      }
      return b.p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    trim(dev);
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{CBFM_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
  }
  return p;
}

void big_release(void* p, size_t bytes, hipStream_t s) {
  int dev = 0;
  hipEvent_t ev = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, s) != hipSuccess) {
    // no way to order a later reuse: wait for the stream, then free
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    return;
  }
  std::vector<Block> drop;
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto& f = cache().free;
    f.push_back({p, bytes, dev, ev});
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
  for (Block& b : drop) {
    (void)hipEventSynchronize(b.ready);
    (void)hipEventDestroy(b.ready);
    (void)hipFree(b.p);
  }
}

}  // namespace cbfm
