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

// Issue-rate probes: every lane runs 8 independent chains of one instruction
// (v_exp_f32 with a negated operand, which keeps the value in (1/2, 1), or an
// FP32 fused multiply-add) so that latency is hidden by the other chains and
// the other wavefronts; the sum of the chains is stored so nothing is elided.
template <int KIND>
__global__ __launch_bounds__(256) void rate_probe_kernel(float* __restrict__ out, int iters) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 0.5f + 0.01f * (float)((threadIdx.x + c) & 7);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (KIND == 0) x[c] = __builtin_amdgcn_exp2f(-x[c]);
      else x[c] = __builtin_fmaf(x[c], 0.999f, 0.0005f);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace crl

extern "C" {

CRL_API int crl_peak_rate(int32_t which, float* scratch, double* per_second, void* stream) {
  if (!scratch || !per_second || (which != CRL_RATE_EXP && which != CRL_RATE_FMA32))
    return CRL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int blocks = CRL_RATE_PROBE_BLOCKS, iters = 4096;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return CRL_EHIP;
  int rc = CRL_OK;
  float best = 0.f;
  for (int rep = 0; rep < 3 && rc == CRL_OK; ++rep) {
    if (hipEventRecord(a, s) != hipSuccess) { rc = CRL_EHIP; break; }
    if (which == CRL_RATE_EXP)
      crl::rate_probe_kernel<0><<<blocks, 256, 0, s>>>(scratch, iters);
    else
      crl::rate_probe_kernel<1><<<blocks, 256, 0, s>>>(scratch, iters);
    if (hipGetLastError() != hipSuccess || hipEventRecord(b, s) != hipSuccess ||
        hipEventSynchronize(b) != hipSuccess) { rc = CRL_EHIP; break; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) { rc = CRL_EHIP; break; }
    if (rep == 0 || ms < best) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != CRL_OK) return rc;
  *per_second = (double)blocks * 256.0 * iters * 8.0 / (best * 1e-3);
  return CRL_OK;
}

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
