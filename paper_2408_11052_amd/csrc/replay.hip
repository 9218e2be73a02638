// The replay buffer as a ring of steps per environment: the insert of a
// chunk of time-major steps and the sampler that relabels goals inside the
// trajectory of the drawn step (gfx950, wave64).
#include "internal.hpp"
#include "relabel.hpp"

namespace crl {

// One wavefront per (step u, env e) row of the chunk: the row's obs and act
// words go to ring row (count + u) mod C of env e, its trajectory id beside
// them.  The chunk is read in order (rows of one step are contiguous), the
// ring is written in whole rows; with V4 (d_s a multiple of 4, both obs
// buffers 16-byte aligned) the obs row moves in 16-byte pieces.
template <bool V4>
__global__ __launch_bounds__(256) void replay_insert_kernel(
    float* __restrict__ obs, float* __restrict__ act, int32_t* __restrict__ traj, int E, int C,
    int d_s, int d_a, const float* __restrict__ nobs, const float* __restrict__ nact,
    const int32_t* __restrict__ ntraj, int U, const int64_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);  // u * E + e
  if (r >= U * E) return;
  const int u = r / E;
  const int e = r - u * E;
  int row = (int)(*count % C) + u;  // u < C, so one wrap at most
  if (row >= C) row -= C;
  const int64_t dst = (int64_t)e * C + row;
  if (V4) {
    float4* __restrict__ so = reinterpret_cast<float4*>(obs + dst * d_s);
    const float4* __restrict__ no = reinterpret_cast<const float4*>(nobs + (int64_t)r * d_s);
    for (int c = lane; c < (d_s >> 2); c += 64) so[c] = no[c];
  } else {
    float* __restrict__ so = obs + dst * d_s;
    const float* __restrict__ no = nobs + (int64_t)r * d_s;
    for (int c = lane; c < d_s; c += 64) so[c] = no[c];
  }
  float* __restrict__ sa = act + dst * d_a;
  const float* __restrict__ na = nact + (int64_t)r * d_a;
  for (int c = lane; c < d_a; c += 64) sa[c] = na[c];
  if (lane == 0) traj[dst] = ntraj[r];
}

// One wavefront per sample.  size = min(count, C) steps are stored, logical
// index i (0 = oldest) at ring row (count - size + i) mod C.  Draw e, i and
// the offset k, then clip i + k to the last step of i's trajectory: the
// lanes compare 64 ids at a time against i's, and the first differing one
// ends the run.  k averages 1 / (1 - gamma), so this is one or two probes of
// 256 contiguous bytes for most samples.
template <typename T>
__global__ __launch_bounds__(256) void ring_relabel_kernel(
    const float* __restrict__ obs, const float* __restrict__ act,
    const int32_t* __restrict__ traj, int E, int C, const int64_t* __restrict__ count,
    int d_s, int d_a, int d_g, int goal_lo, uint64_t seed, const int64_t* __restrict__ step,
    const uint64_t* __restrict__ thr, int n_thr, int B, int32_t* __restrict__ idx,
    T* __restrict__ x_sa, int ld_sa, T* __restrict__ x_g, int ld_g,
    T* __restrict__ x_sg, int ld_sg) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  const int64_t cnt = *count;
  const int size = (int)(cnt < (int64_t)C ? cnt : (int64_t)C);
  if (size < 2) {  // nothing to draw: (-1, -1, -1) and zero rows
    if (lane == 0) {
      idx[3 * b + 0] = -1;
      idx[3 * b + 1] = -1;
      idx[3 * b + 2] = -1;
    }
    write_inputs<T>(nullptr, nullptr, nullptr, d_s, d_a, d_g, b, lane, x_sa, ld_sa, x_g, ld_g,
                    x_sg, ld_sg);
    return;
  }
  const GeomProbe probe = geom_prefetch(thr, n_thr, lane);
  const int base = (int)((cnt - size) % C);  // ring row of logical index 0
  uint64_t x[4] = {(uint64_t)b, (uint64_t)(*step), 0ull, 0ull};
  philox4x64_10(x, seed, 0ull);
  const int e = (int)__umul64hi(x[0], (uint64_t)E);
  const int i = (int)__umul64hi(x[1], (uint64_t)(size - 1));
  const int km1 = geom_count(thr, probe, x[2], lane);  // k - 1
  const int32_t* __restrict__ tr = traj + (int64_t)e * C;
  auto ring_row = [&](int j) { int q = base + j; return q >= C ? q - C : q; };
  const int32_t tid = tr[ring_row(i)];
  const int lim = min(i + 1 + km1, size - 1);
  int tg = lim;
  for (int j0 = i + 1; j0 <= lim; j0 += 64) {
    const int j = j0 + lane;
    const bool other = j <= lim && tr[ring_row(j)] != tid;
    const uint64_t m = __ballot(other);
    if (m) {
      tg = j0 + (int)__builtin_ctzll(m) - 1;
      break;
    }
  }
  const int ri = ring_row(i), rg = ring_row(tg);
  if (lane == 0) {
    idx[3 * b + 0] = e;
    idx[3 * b + 1] = ri;
    idx[3 * b + 2] = rg;
  }
  const float* s_row = obs + ((int64_t)e * C + ri) * d_s;
  const float* a_row = act + ((int64_t)e * C + ri) * d_a;
  const float* g_row = obs + ((int64_t)e * C + rg) * d_s + goal_lo;
  write_inputs<T>(s_row, a_row, g_row, d_s, d_a, d_g, b, lane, x_sa, ld_sa, x_g, ld_g, x_sg,
                  ld_sg);
}

hipError_t launch_replay_insert(float* obs, float* act, int32_t* traj, int E, int C, int d_s,
                                int d_a, const float* nobs, const float* nact,
                                const int32_t* ntraj, int U, int64_t* count, hipStream_t s) {
  const int64_t rows = (int64_t)U * E;
  dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  const double bytes = 2.0 * (double)rows * (4.0 * (d_s + d_a) + 4.0);
  const bool v4 = (d_s & 3) == 0 && ((reinterpret_cast<uintptr_t>(obs) |
                                       reinterpret_cast<uintptr_t>(nobs)) & 15u) == 0;
  if (v4)
    CRL_TIMED("replay_insert_kernel", 0.0, bytes, s,
      replay_insert_kernel<true><<<grid, block, 0, s>>>(obs, act, traj, E, C, d_s, d_a, nobs,
                                                        nact, ntraj, U, count));
  else
    CRL_TIMED("replay_insert_kernel", 0.0, bytes, s,
      replay_insert_kernel<false><<<grid, block, 0, s>>>(obs, act, traj, E, C, d_s, d_a, nobs,
                                                         nact, ntraj, U, count));
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_counter_add(count, U, s);
}

hipError_t launch_ring_relabel(const float* obs, const float* act, const int32_t* traj, int E,
                               int C, const int64_t* count, int d_s, int d_a, int d_g,
                               int goal_lo, uint64_t seed, const int64_t* step,
                               const uint64_t* thr, int n_thr, int B, int32_t* idx, void* x_sa,
                               int ld_sa, void* x_g, int ld_g, void* x_sg, int ld_sg, bool bf16,
                               hipStream_t s) {
  dim3 grid((B + 3) / 4), block(256);
  const double es = bf16 ? 2.0 : 4.0;
  const double bytes = (double)B * (4.0 * (d_s + d_a + d_g + (x_sg ? d_s + d_g : 0)) +
                                    es * (ld_sa + ld_g + (x_sg ? ld_sg : 0)) + 12.0);
  if (bf16)
    CRL_TIMED("ring_relabel_kernel", 0.0, bytes, s,
      ring_relabel_kernel<bf16_t><<<grid, block, 0, s>>>(obs, act, traj, E, C, count, d_s, d_a,
        d_g, goal_lo, seed, step, thr, n_thr, B, idx, (bf16_t*)x_sa, ld_sa, (bf16_t*)x_g, ld_g,
        (bf16_t*)x_sg, ld_sg));
  else
    CRL_TIMED("ring_relabel_kernel", 0.0, bytes, s,
      ring_relabel_kernel<float><<<grid, block, 0, s>>>(obs, act, traj, E, C, count, d_s, d_a,
        d_g, goal_lo, seed, step, thr, n_thr, B, idx, (float*)x_sa, ld_sa, (float*)x_g, ld_g,
        (float*)x_sg, ld_sg));
  return hipGetLastError();
}

}  // namespace crl
