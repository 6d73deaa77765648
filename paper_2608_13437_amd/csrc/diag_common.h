// Block reductions of the diagnostic partial sums (device side).
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"

namespace cnsf {

__device__ inline void part_zero(DiagPartial& p) {
  p.mass = p.mx = p.my = p.mz = p.energy = p.ek2 = 0.0;
  p.min_rho = p.min_p = 1e300;
  p.sensor = p.nonfinite = 0.0;
  p.eps_s = p.eps_d = 0.0;
}

__device__ inline void part_add(DiagPartial& a, const DiagPartial& b) {
  a.mass += b.mass;
  a.mx += b.mx;
  a.my += b.my;
  a.mz += b.mz;
  a.energy += b.energy;
  a.ek2 += b.ek2;
  a.min_rho = fmin(a.min_rho, b.min_rho);
  a.min_p = fmin(a.min_p, b.min_p);
  a.sensor += b.sensor;
  a.nonfinite += b.nonfinite;
  a.eps_s += b.eps_s;
  a.eps_d += b.eps_d;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  return v;
}

// Block total of one DiagPartial per thread (wave shuffles, then the wave
// results in index order; blockDim.x a multiple of 64, at most 256); valid in
// thread 0.  Deterministic.
__device__ inline DiagPartial block_reduce(DiagPartial v) {
  __shared__ DiagPartial sh[4];
  v.mass = wave_sum(v.mass);
  v.mx = wave_sum(v.mx);
  v.my = wave_sum(v.my);
  v.mz = wave_sum(v.mz);
  v.energy = wave_sum(v.energy);
  v.ek2 = wave_sum(v.ek2);
  v.min_rho = wave_min(v.min_rho);
  v.min_p = wave_min(v.min_p);
  v.sensor = wave_sum(v.sensor);
  v.nonfinite = wave_sum(v.nonfinite);
  v.eps_s = wave_sum(v.eps_s);
  v.eps_d = wave_sum(v.eps_d);
  const int w = threadIdx.x / 64, nw = blockDim.x / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  DiagPartial t = sh[0];
  for (int i = 1; i < nw; ++i) part_add(t, sh[i]);
  return t;
}

// The Eq. (7) sums of one cell from its gathered (shifted, FP32 or 16-bit)
// populations: moments summed in FP64 from the stored values, FP64
// primitives; optionally u, v, w, mu into the spectral fields.
template <typename Gf>
__device__ inline void cell_sums(const Gf& gf, const Codec& cd, const PhysD& phd, uint32_t c, uint64_t ncells,
                                 double* __restrict__ fields, DiagPartial& acc) {
  double Q[NC];
  bool finite = true;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) s += (double)gf[k][i];
    Q[k] = q_ref<double>(cd, k) + s;
    finite = finite && isfinite(s);
  }
  Prim<double> P = primitives<double>(Q, phd);
  acc.mass += Q[0];
  acc.mx += Q[1];
  acc.my += Q[2];
  acc.mz += Q[3];
  acc.energy += Q[4];
  acc.ek2 += Q[1] * P.u[0] + Q[2] * P.u[1] + Q[3] * P.u[2];
  acc.min_rho = fmin(acc.min_rho, P.rho);
  acc.min_p = fmin(acc.min_p, P.p);
  acc.nonfinite += finite ? 0.0 : 1.0;
  if (fields) {
    fields[c] = P.u[0];
    fields[ncells + c] = P.u[1];
    fields[2 * ncells + c] = P.u[2];
    fields[3 * ncells + c] = P.muT;
  }
}

}  // namespace cnsf
