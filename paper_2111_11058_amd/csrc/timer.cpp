// Opt-in launch timing with HIP events (cbfm_timer_enable / cbfm_timer_read).
#include <cstring>
#include <mutex>

#include "internal.h"

namespace cbfm {

namespace {
std::mutex g_mu;
uint32_t g_mask = 0;  // bit i: kernel family i is timed
struct Pending {
  hipEvent_t e0, e1;
  double work;
};
struct Rec {
  std::vector<Pending> pending;
  int64_t launches = 0;
  double ms = 0, work = 0;
};
Rec g_rec[T_COUNT];
const char* g_names[T_COUNT] = {"fill_regular", "fill_near",    "assemble",         "gemm",      "gmres_dots",
                                "gmres_update", "fill_regular_f32", "xgemm",        "gemm_panel"};

void drain(Rec& r) {
  for (auto& p : r.pending) {
    float ms = 0;
    if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      r.ms += ms;
      r.launches += 1;
      r.work += p.work;
    }
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  r.pending.clear();
}
}  // namespace

TimedLaunch::TimedLaunch(int id_, hipStream_t s_, double work_) : id(id_), s(s_), work(work_) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!(g_mask >> id & 1u)) return;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone) return;  // no events in graphs
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}

TimedLaunch::~TimedLaunch() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_mu);
  g_rec[id].pending.push_back({e0, e1, work});
}

}  // namespace cbfm

using namespace cbfm;

extern "C" cbfm_status cbfm_timer_enable(int32_t mask) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_rec) {
      drain(r);
      r.launches = 0;
      r.ms = 0;
      r.work = 0;
    }
    g_mask = (uint32_t)mask;
  });
}

extern "C" cbfm_status cbfm_timer_read(const char* name, int64_t* launches, double* total_ms, double* work) {
  return guarded([&] {
    CBFM_REQUIRE(name != nullptr, CBFM_E_ARG, "timer name is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    for (int i = 0; i < T_COUNT; ++i)
      if (std::strcmp(name, g_names[i]) == 0) {
        drain(g_rec[i]);
        if (launches) *launches = g_rec[i].launches;
        if (total_ms) *total_ms = g_rec[i].ms;
        if (work) *work = g_rec[i].work;
        return;
      }
    throw Error{CBFM_E_ARG, std::string("unknown timer ") + name};
  });
}
