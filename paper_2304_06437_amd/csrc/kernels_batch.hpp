// Batched sweeps: many independent simulations of one kernel configuration
// advanced by a single launch per sweep.
//
// The launch's work units (blocks for the moments sweep, wavefronts for
// stream-collide) are numbered consecutively across the jobs; a job
// descriptor table, sorted by first unit, maps a unit to its job by binary
// search.  Each unit then runs exactly the per-unit code of the single-job
// kernels, so a job's result does not depend on what else is in the batch.
#pragma once

#include "kernels.hpp"
#include "kernels2.hpp"

namespace lbk {

template <typename C>
struct JobDesc {
  StepParams<C> p;
  ColourParams<C> cp;
  const void* m;   // moment arrays (compute type)
  void* f;         // population arrays (storage type)
  int64_t start;   // first work unit of this job in the launch
};

// Last job whose first unit is <= u (jobs sorted by start, jobs[0].start = 0).
template <typename C>
__device__ __forceinline__ int job_of(const JobDesc<C>* __restrict__ jobs, int njobs, int64_t u) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].start <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class L, int SPECIES, typename S, typename C, int V>
__global__ __launch_bounds__(256) void k_moments_batch(const JobDesc<C>* __restrict__ jobs,
                                                       int njobs, int64_t total) {
  const int64_t u = flat_block();
  if (u >= total) return;  // block-uniform
  const JobDesc<C>& J = jobs[job_of(jobs, njobs, u)];
  const int64_t i0 = ((u - J.start) * blockDim.x + threadIdx.x) * V;
  if constexpr (SPECIES == 1)
    moments_body<L, S, C, V>((const S*)J.f, (C*)J.m, J.p, i0);
  else
    moments2_body<L, S, C, V>((const S*)J.f, (C*)J.m, J.p, J.cp, i0);
}

template <class L, int ORDER, int SPECIES, typename S, typename C, int E, int H, bool FD = false>
__global__ __launch_bounds__(256) void k_stream_collide_batch(const JobDesc<C>* __restrict__ jobs,
                                                              int njobs, int64_t total) {
  const int64_t w = flat_block() * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= total) return;  // wave-uniform
  const JobDesc<C>& J = jobs[job_of(jobs, njobs, w)];
  if constexpr (SPECIES == 1)
    // the padded-row variant: jobs with and without padded rows share a launch
    StreamCollide<L, ORDER, S, C, E, H, FD, true>::run_wave((const C*)J.m, (S*)J.f, J.p,
                                                            w - J.start);
  else
    StreamCollide2<L, S, C, E>::run_wave((const C*)J.m, (S*)J.f, J.p, J.cp, w - J.start);
}

}  // namespace lbk
