// Opt-in per-kernel timing: HIP events recorded on the launch stream around
// each kernel launch, grouped by kernel name, with the algorithmic FLOPs and
// HBM bytes of each launch.  Off by default; never records while the stream
// is being captured into a graph.
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "crl.h"
#include "internal.hpp"

namespace crl {
namespace {

struct Slot {
  std::string name;
  int64_t launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Slot> g_slots;
std::map<std::string, int> g_index;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Drain pending pairs of every slot into its millisecond total.
hipError_t drain_locked() {
  for (Slot& s : g_slots) {
    for (auto& pr : s.pending) {
      hipError_t e = hipEventSynchronize(pr.second);
      if (e != hipSuccess) return e;
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, pr.first, pr.second);
      if (e != hipSuccess) return e;
      s.ms += ms;
      g_pool.push_back(pr.first);
      g_pool.push_back(pr.second);
    }
    s.pending.clear();
  }
  return hipSuccess;
}

}  // namespace

KTimer timing_begin(const char* name, double flops, double bytes, hipStream_t s) {
  KTimer t{};
  t.on = false;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return t;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return t;
  auto it = g_index.find(name);
  int slot;
  if (it == g_index.end()) {
    slot = (int)g_slots.size();
    g_slots.emplace_back();
    g_slots.back().name = name;
    g_index[name] = slot;
  } else {
    slot = it->second;
  }
  t.a = take_event();
  t.b = take_event();
  if (!t.a || !t.b) return t;
  if (hipEventRecord(t.a, s) != hipSuccess) return t;
  t.slot = slot;
  t.s = s;
  t.flops = flops;
  t.bytes = bytes;
  t.on = true;
  return t;
}

void timing_end(KTimer& t) {
  if (!t.on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(t.b, t.s) != hipSuccess) return;
  Slot& s = g_slots[t.slot];
  s.launches += 1;
  s.flops += t.flops;
  s.bytes += t.bytes;
  s.pending.emplace_back(t.a, t.b);
  t.on = false;
}

}  // namespace crl

extern "C" {

CRL_API int crl_timing_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(crl::g_mu);
  crl::g_on = enable != 0;
  return CRL_OK;
}

CRL_API int crl_timing_reset(void) {
  std::lock_guard<std::mutex> lk(crl::g_mu);
  hipError_t e = crl::drain_locked();
  crl::g_slots.clear();
  crl::g_index.clear();
  return e == hipSuccess ? CRL_OK : CRL_EHIP;
}

CRL_API int crl_timing_count(int32_t* n) {
  if (!n) return CRL_EINVAL;
  std::lock_guard<std::mutex> lk(crl::g_mu);
  *n = (int32_t)crl::g_slots.size();
  return CRL_OK;
}

CRL_API int crl_timing_read(int32_t i, char* name, int32_t name_len, int64_t* launches,
                            double* ms, double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(crl::g_mu);
  if (i < 0 || i >= (int32_t)crl::g_slots.size()) return CRL_EINVAL;
  if (crl::drain_locked() != hipSuccess) return CRL_EHIP;
  const crl::Slot& s = crl::g_slots[i];
  if (name && name_len > 0) {
    size_t n = s.name.size() < (size_t)(name_len - 1) ? s.name.size() : (size_t)(name_len - 1);
    s.name.copy(name, n);
    name[n] = '\0';
  }
  if (launches) *launches = s.launches;
  if (ms) *ms = s.ms;
  if (flops) *flops = s.flops;
  if (bytes) *bytes = s.bytes;
  return CRL_OK;
}

}  // extern "C"
