// The geometric goal offset shared by the episode-row and ring samplers.
#pragma once

#include "common.hpp"

namespace crl {

// First level of the threshold search, issued before Philox runs: the probes
// of the first level are the same 64 entries for every sample.
struct GeomProbe {
  int n_thr, step0, q0;
  uint64_t thr0;
};
__device__ inline GeomProbe geom_prefetch(const uint64_t* __restrict__ thr, int n_thr, int lane) {
  GeomProbe p;
  p.n_thr = n_thr;
  p.step0 = (n_thr + 63) >> 6;
  p.q0 = lane * p.step0;
  p.thr0 = (n_thr > 64 && p.q0 < n_thr) ? thr[p.q0] : 0ull;
  return p;
}

// k - 1 = #{m in [1, n_thr] : w2 < thr[m]} (thr[m] stored at index m - 1).
// The table is non-increasing, so the count is the length of its prefix that
// exceeds w2.  64-way search: the lanes probe 64 evenly spaced entries of the
// remaining range at once, and the number of probes above w2 narrows the
// prefix end to one gap between probes.  Every lane of the wave must call it
// with the same w2; every lane returns the same count.
__device__ inline int geom_count(const uint64_t* __restrict__ thr, const GeomProbe& p,
                                 uint64_t w2, int lane) {
  int lo = 0, hi = p.n_thr;  // count in [lo, hi]
  if (hi - lo > 64) {
    const bool above = p.q0 < hi && p.thr0 > w2;
    const int c = __popcll(__ballot(above));
    const int nlo = c > 0 ? (c - 1) * p.step0 + 1 : 0;
    hi = min(hi, c * p.step0);
    lo = nlo;
  }
  while (hi - lo > 64) {
    const int step = (hi - lo + 63) >> 6;
    const int q = lo + lane * step;
    const bool above = q < hi && thr[q] > w2;
    const int c = __popcll(__ballot(above));  // probes 0..c-1 are above w2
    const int nlo = c > 0 ? lo + (c - 1) * step + 1 : lo;
    const int qc = lo + c * step;             // first probe not above (or past hi)
    hi = min(hi, qc);
    lo = nlo;
  }
  const int q = lo + lane;
  const bool above = q < hi && thr[q] > w2;
  return lo + __popcll(__ballot(above));
}

// One sample's encoder inputs from its rows (one wavefront, lane-strided):
// x_sa = [s, a, 0...], x_g = [g, 0...], x_sg = [s, g, 0...] (x_sg optional).
// With s_row == nullptr every column is 0 (no sample could be drawn).
template <typename T>
__device__ inline void write_inputs(const float* s_row, const float* a_row, const float* g_row,
                                    int d_s, int d_a, int d_g, int64_t b, int lane,
                                    T* __restrict__ x_sa, int ld_sa, T* __restrict__ x_g, int ld_g,
                                    T* __restrict__ x_sg, int ld_sg) {
  const bool ok = s_row != nullptr;
  for (int c = lane; c < ld_sa; c += 64) {
    float v = 0.f;
    if (ok) v = c < d_s ? s_row[c] : (c < d_s + d_a ? a_row[c - d_s] : 0.f);
    x_sa[b * ld_sa + c] = Store<T>::from_f(v);
  }
  for (int c = lane; c < ld_g; c += 64)
    x_g[b * ld_g + c] = Store<T>::from_f(ok && c < d_g ? g_row[c] : 0.f);
  if (x_sg) {
    for (int c = lane; c < ld_sg; c += 64) {
      float v = 0.f;
      if (ok) v = c < d_s ? s_row[c] : (c < d_s + d_g ? g_row[c - d_s] : 0.f);
      x_sg[b * ld_sg + c] = Store<T>::from_f(v);
    }
  }
}

}  // namespace crl
