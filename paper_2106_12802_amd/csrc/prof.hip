// Per-kernel timing with HIP events recorded on the launch stream.
#include <utility>
#include <vector>

#include "mrs_internal.hpp"

namespace mrs {
namespace {

struct Pending {
  int id;
  hipEvent_t start, stop;
};

bool g_on = false;
thread_local int t_paused = 0;  // ProfPause scopes open on this thread
uint32_t g_mask = 0xffffffffu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
hipEvent_t g_open[MRS_NUM_KERNEL_IDS] = {};
double g_ms[MRS_NUM_KERNEL_IDS] = {};
int64_t g_count[MRS_NUM_KERNEL_IDS] = {};

hipEvent_t take() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void drain() {
  for (auto& p : g_pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      g_ms[p.id] += ms;
      g_count[p.id] += 1;
    } else {
      (void)hipGetLastError();
    }
    g_free.push_back(p.start);
    g_free.push_back(p.stop);
  }
  g_pending.clear();
}

}  // namespace

ProfPause::ProfPause() { ++t_paused; }
ProfPause::~ProfPause() { --t_paused; }

void prof_begin(int id, hipStream_t st) {
  if (!g_on || t_paused || id < 0 || id >= MRS_NUM_KERNEL_IDS || !((g_mask >> id) & 1u)) return;
  hipEvent_t e = take();
  if (e && hipEventRecord(e, st) == hipSuccess) {
    g_open[id] = e;
  } else {
    (void)hipGetLastError();
    if (e) g_free.push_back(e);
    g_open[id] = nullptr;
  }
}

void prof_end(int id, hipStream_t st) {
  if (!g_on || t_paused || id < 0 || id >= MRS_NUM_KERNEL_IDS || !g_open[id]) return;
  hipEvent_t e = take();
  if (e && hipEventRecord(e, st) == hipSuccess) {
    g_pending.push_back({id, g_open[id], e});
  } else {
    (void)hipGetLastError();
    g_free.push_back(g_open[id]);
    if (e) g_free.push_back(e);
  }
  g_open[id] = nullptr;
  if (g_pending.size() > 8192) {  // bound the number of live events
    (void)hipDeviceSynchronize();
    drain();
  }
}

mrs_status prof_enable(bool on) {
  if (!g_pending.empty()) {
    MRS_TRY_HIP(hipDeviceSynchronize());
    g_pending.clear();  // discard: totals restart
  }
  for (int i = 0; i < MRS_NUM_KERNEL_IDS; ++i) {
    g_ms[i] = 0.0;
    g_count[i] = 0;
    g_open[i] = nullptr;
  }
  g_on = on;
  return MRS_OK;
}

mrs_status prof_select(uint32_t mask) {
  g_mask = mask;
  return MRS_OK;
}

mrs_status prof_read(double* ms, int64_t* launches) {
  MRS_TRY_HIP(hipDeviceSynchronize());
  drain();
  for (int i = 0; i < MRS_NUM_KERNEL_IDS; ++i) {
    ms[i] = g_ms[i];
    launches[i] = g_count[i];
  }
  return MRS_OK;
}

}  // namespace mrs
