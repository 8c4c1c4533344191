// Fence-free grid reductions.  A kernel leaves one partial record per
// workgroup (plain stores); the kernel that consumes the total adds the
// records up itself, every workgroup in the same fixed order, so the result
// is identical everywhere and deterministic.  Kernel boundaries order the
// stores before the loads.  (The alternative, a last-workgroup reduction,
// needs a device-scope fence in every workgroup, which writes back the
// XCD's L2 each time.)
#pragma once

#include "common.hpp"

namespace qsp {
namespace partials {

// Workgroup sums of v stored at part[bid * NV + k].
template <int NV>
__device__ inline void store(double (&v)[NV], double* part, int bid) {
  __shared__ double red[NV][kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) s += red[k][w];
      part[static_cast<size_t>(bid) * NV + k] = s;
    }
}

// Totals of nblk partial records; every thread of the workgroup gets them.
template <int NV>
__device__ inline void sum(const double* part, int nblk, double (&tot)[NV]) {
  __shared__ double red[NV][kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double t[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) t[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] += part[static_cast<size_t>(b) * NV + k];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int off = 32; off > 0; off >>= 1) t[k] += __shfl_down(t[k], off, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wave] = t[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[k][w];
    tot[k] = s;
  }
  __syncthreads();   // red may be reused by the caller's next reduction
}

// Predictor-corrector convergence test of the last corrector solve, from
// its partial records (|B_new - B_old|^2, |B_new|^2): relative change
// sqrt(sum d / sum s) against tol.  Every workgroup gets the decision; the
// one with `record` set books it (residual, iteration count, done flag).
__device__ inline bool pc_consume(const double* part, int nblk, double tol, DevCounters* ctr,
                                  bool record) {
  double t[2];
  sum<2>(part, nblk, t);
  const double dd = t[0], ss = t[1];
  const double res = ss > 0.0 ? sqrt(dd / ss) : (dd == 0.0 ? 0.0 : INFINITY);
  const bool done = tol > 0.0 && res < tol;
  if (record && threadIdx.x == 0) {
    if (!isfinite(res) || !isfinite(dd) || !isfinite(ss)) ctr->nonfinite = 1u;
    ctr->pc_resid = res;
    ctr->pc_iters += 1u;
    ctr->pc_iterations += 1ull;
    if (done) ctr->pc_done = 1u;
  }
  return done;
}

}  // namespace partials
}  // namespace qsp
