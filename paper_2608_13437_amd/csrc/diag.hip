// FP64 diagnostics of the current time level (Eq. (7), Section 3.2).
//
// Pass 1 (sums): per cell, decode the populations, form Q, primitives and
// mu_T, accumulate mass, momentum, energy, rho |u|^2, minima, non-finite and
// sensor-active counts into one partial per block (fixed grid, grid-stride),
// and optionally write u, v, w, mu_T to the spectral workspace.
// Passes 2-4 (spectral): for each axis, every line of the periodic box is
// transformed in LDS (radix-2 FFT for power-of-two lengths, otherwise a
// direct sum with the trigonometric-interpolant derivative kernel), multiplied
// by i k (the Nyquist mode of an even length differentiates to zero) and
// transformed back; derivatives accumulate into div u and curl u.  The last
// axis also reduces mu |curl u|^2 and mu (div u)^2 into the block partials.
// Pass 5 reduces the block partials in a fixed order (deterministic).
#include "cnsf_impl.h"
#include "launch.h"

namespace cnsf {

constexpr int DB = 256;  // threads per diagnostics block

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

// Block total of one DiagPartial per thread (wave shuffles, then the DB/64
// wave results in index order); valid in thread 0.  Deterministic.
__device__ inline DiagPartial block_reduce(DiagPartial v) {
  __shared__ DiagPartial sh[DB / 64];
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
  const int w = threadIdx.x / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  DiagPartial t = sh[0];
  for (int i = 1; i < DB / 64; ++i) part_add(t, sh[i]);
  return t;
}

template <int ST, int BC>
__global__ void __launch_bounds__(DB) k_diag_sums(const typename Store<ST>::T* __restrict__ pop, const Geom g,
                                                  const Phys ph, const PhysD phd, const Codec cd, int parity,
                                                  DiagPartial* __restrict__ partials, double* __restrict__ fields) {
  DiagPartial acc;
  part_zero(acc);
  const uint32_t stride = gridDim.x * DB;
  for (uint32_t c = blockIdx.x * DB + threadIdx.x; c < g.ncells; c += stride) {
    const Nbr n = neighbours(c, g);
    uint32_t off[NV];
    stream_offsets<ST, BC>(g, n, parity, off);
    double gv[NC][NV];
    gather<ST, BC, true, double>(pop, g, cd, n, parity, off, gv);
    double Q[NC];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i) s += gv[k][i];
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
    // the sensor decision as the FP32 update takes it
    float gf[NC][NV], dQf[NC], Qf[NC];
    DevPrim Pf;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int i = 0; i < NV; ++i) gf[k][i] = (float)gv[k][i];
    float chi = 0.0f;
    cell_state(gf, cd, ph, dQf, Qf, Pf, &chi);
    acc.sensor += chi > 0.0f ? 1.0 : 0.0;
    if (fields) {
      const uint64_t N = g.ncells;
      fields[c] = P.u[0];
      fields[N + c] = P.u[1];
      fields[2 * N + c] = P.u[2];
      fields[3 * N + c] = P.muT;
    }
  }
  DiagPartial tot = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// ------------------------------------------------------------------ spectral
struct AxisGeom {
  uint32_t n;        // line length
  uint32_t stride;   // element stride along the line
  uint32_t nlines;
  uint32_t lines_per_block;
  uint32_t log2n;    // 0 if n is not a power of two
  int axis;          // 0 x, 1 y, 2 z
  int last;          // reduce eps into the partials
  double kscale;     // 2 pi / (n dx)
};

__device__ inline uint32_t line_base(uint32_t l, int axis, const Geom& g) {
  if (axis == 0) return l * g.nx;                       // l = y + ny z
  if (axis == 1) return (l / g.nx) * g.nxy + (l % g.nx);  // l = x + nx z
  return l;                                             // l = x + nx y
}

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// In-place radix-2 transform of `cnt` lines of length n held in LDS, bit-reversed
// input (forward, DIT) or natural input (inverse, DIF).  sign = -1 forward, +1 inverse.
__device__ inline void fft_dit(double2* buf, uint32_t n, uint32_t log2n, uint32_t cnt) {
  const uint32_t half = n / 2;
  for (uint32_t h = 1; h < n; h <<= 1) {
    for (uint32_t t = threadIdx.x; t < cnt * half; t += blockDim.x) {
      const uint32_t line = t / half, b = t % half;
      const uint32_t m = b % h, j = (b / h) * 2 * h + m;
      double s, c;
      sincospi(-(double)m / (double)h, &s, &c);
      double2* L = buf + line * n;
      const double2 x0 = L[j], x1 = cmul(make_double2(c, s), L[j + h]);
      L[j] = make_double2(x0.x + x1.x, x0.y + x1.y);
      L[j + h] = make_double2(x0.x - x1.x, x0.y - x1.y);
    }
    __syncthreads();
  }
}

__device__ inline void fft_dif_inv(double2* buf, uint32_t n, uint32_t log2n, uint32_t cnt) {
  const uint32_t half = n / 2;
  for (uint32_t h = half; h >= 1; h >>= 1) {
    for (uint32_t t = threadIdx.x; t < cnt * half; t += blockDim.x) {
      const uint32_t line = t / half, b = t % half;
      const uint32_t m = b % h, j = (b / h) * 2 * h + m;
      double s, c;
      sincospi((double)m / (double)h, &s, &c);
      double2* L = buf + line * n;
      const double2 x0 = L[j], x1 = L[j + h];
      L[j] = make_double2(x0.x + x1.x, x0.y + x1.y);
      L[j + h] = cmul(make_double2(x0.x - x1.x, x0.y - x1.y), make_double2(c, s));
    }
    __syncthreads();
  }
}

// Derivatives along one axis of u, v, w for a group of lines; accumulate into
// div u and curl u:  omega_c = eps_{c a b} d_a u_b.
__global__ void __launch_bounds__(DB) k_spectral_axis(double* __restrict__ fields, const Geom g, const AxisGeom ag,
                                                      DiagPartial* __restrict__ partials) {
  extern __shared__ double2 lds[];
  const uint32_t n = ag.n, TL = ag.lines_per_block;
  const uint64_t N = g.ncells;
  const double* u[3] = {fields, fields + N, fields + 2 * N};
  const double* mu = fields + 3 * N;
  double* divf = fields + 4 * N;
  double* wf[3] = {fields + 5 * N, fields + 6 * N, fields + 7 * N};
  const int a = ag.axis;
  const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;  // eps_{b2 a b1} = +1, eps_{b1 a b2} = -1
  const bool pow2 = ag.log2n != 0;
  double2* A = lds;            // u_a + i u_b1
  double2* B = lds + TL * n;   // u_b2 + i 0
  // direct path (non power of two): separate output rows and the derivative kernel
  double2* Aout = pow2 ? A : lds + 2 * TL * n;
  double2* Bout = pow2 ? B : lds + 3 * TL * n;
  double* Dk = (double*)(lds + (pow2 ? 2 : 4) * TL * n);
  if (!pow2) {
    // D[m] = -(2/n) sum_{k=1}^{K} kappa_k sin(2 pi k m / n), Nyquist excluded
    const uint32_t K = (n % 2) ? (n - 1) / 2 : n / 2 - 1;
    for (uint32_t m = threadIdx.x; m < n; m += blockDim.x) {
      double sacc = 0.0;
      for (uint32_t k = 1; k <= K; ++k) sacc += (double)k * sinpi(2.0 * (double)((uint64_t)k * m % n) / (double)n);
      Dk[m] = -2.0 / (double)n * ag.kscale * sacc;
    }
  }
  DiagPartial acc;
  part_zero(acc);
  const uint32_t groups = (ag.nlines + TL - 1) / TL;
  for (uint32_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    const uint32_t l0 = grp * TL;
    const uint32_t cnt = min(TL, ag.nlines - l0);
    __syncthreads();
    // load (bit-reversed positions for the decimation-in-time transform)
    for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
      uint32_t line, j;
      if (a == 0) { line = e / n; j = e % n; }
      else { line = e % cnt; j = e / cnt; }
      const uint32_t addr = line_base(l0 + line, a, g) + j * ag.stride;
      const uint32_t pos = pow2 ? (__brev(j) >> (32 - ag.log2n)) : j;
      A[line * n + pos] = make_double2(u[a][addr], u[b1][addr]);
      B[line * n + pos] = make_double2(u[b2][addr], 0.0);
    }
    __syncthreads();
    if (pow2) {
      fft_dit(A, n, ag.log2n, cnt);
      fft_dit(B, n, ag.log2n, cnt);
      // multiply by i kappa_j (Nyquist to zero) and 1/n for the inverse
      for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
        const uint32_t j = e % n;
        double kj = (j < n / 2) ? (double)j : (j == n / 2 ? 0.0 : (double)j - (double)n);
        kj *= ag.kscale / (double)n;
        const double2 x = A[e], y = B[e];
        A[e] = make_double2(-kj * x.y, kj * x.x);
        B[e] = make_double2(-kj * y.y, kj * y.x);
      }
      __syncthreads();
      fft_dif_inv(A, n, ag.log2n, cnt);   // output in bit-reversed positions
      fft_dif_inv(B, n, ag.log2n, cnt);
    } else {
      // direct: d_j = sum_m D[m] x_{(j - m) mod n}
      for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
        const uint32_t line = e / n, j = e % n;
        double da = 0.0, db1 = 0.0, db2 = 0.0;
        for (uint32_t m = 0; m < n; ++m) {
          const uint32_t src = line * n + (j + n - m) % n;
          const double d = Dk[m];
          da += d * A[src].x;
          db1 += d * A[src].y;
          db2 += d * B[src].x;
        }
        Aout[e] = make_double2(da, db1);
        Bout[e] = make_double2(db2, 0.0);
      }
      __syncthreads();
    }
    // write / accumulate
    for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
      uint32_t line, j;
      if (a == 0) { line = e / n; j = e % n; }
      else { line = e % cnt; j = e / cnt; }
      const uint32_t addr = line_base(l0 + line, a, g) + j * ag.stride;
      const uint32_t pos = pow2 ? (__brev(j) >> (32 - ag.log2n)) : j;
      const double2 ra = Aout[line * n + pos];
      const double dua = ra.x, dub1 = ra.y, dub2 = Bout[line * n + pos].x;
      // omega_{b2} += d_a u_{b1};  omega_{b1} -= d_a u_{b2}
      double dv = dua;
      const double wb2 = dub1, wb1 = -dub2;
      if (a == 0) {        // first pass: div, omega_z (b2 = 2), omega_y (b1 = 1)
        divf[addr] = dv;
        wf[b2][addr] = wb2;
        wf[b1][addr] = wb1;
      } else if (a == 1) { // omega_x (b2 = 0) starts here; omega_z (b1 = 2) accumulates
        divf[addr] += dv;
        wf[b2][addr] = wb2;
        wf[b1][addr] += wb1;
      } else {             // last pass: b1 = 0 (omega_x), b2 = 1 (omega_y); reduce
        dv += divf[addr];
        const double wx = wf[0][addr] + wb1;
        const double wy = wf[1][addr] + wb2;
        const double wz = wf[2][addr];
        const double m = mu[addr];
        acc.eps_s += m * (wx * wx + wy * wy + wz * wz);
        acc.eps_d += m * dv * dv;
      }
    }
  }
  if (ag.last) {
    DiagPartial tot = block_reduce(acc);
    if (threadIdx.x == 0) {
      partials[blockIdx.x].eps_s = tot.eps_s;
      partials[blockIdx.x].eps_d = tot.eps_d;
    }
  }
}

__global__ void k_diag_final(const DiagPartial* __restrict__ partials, int nparts, DiagPartial* __restrict__ out) {
  DiagPartial acc;
  part_zero(acc);
  for (int i = threadIdx.x; i < nparts; i += DB) part_add(acc, partials[i]);
  DiagPartial tot = block_reduce(acc);
  if (threadIdx.x == 0) *out = tot;
}

// ------------------------------------------------------------------ launchers
template <int ST, int BC>
static hipError_t diag_sums_t(const void* pop, const Geom& g, const Phys& ph, const PhysD& phd, const Codec& cd,
                              int parity, DiagPartial* partials, double* fields, hipStream_t s) {
  hipLaunchKernelGGL((k_diag_sums<ST, BC>), dim3(DIAG_BLOCKS), dim3(DB), 0, s, (const typename Store<ST>::T*)pop, g, ph,
                     phd, cd, parity, partials, fields);
  return hipGetLastError();
}

hipError_t launch_diag_sums(int storage, const void* pop, const Geom& g, const Phys& ph, const PhysD& phd,
                            const Codec& cd, int parity, DiagPartial* partials, double* fields, hipStream_t s) {
#define CNSF_CASE(ST, BC) \
  if (storage == ST && g.bc_x == BC) return diag_sums_t<ST, BC>(pop, g, ph, phd, cd, parity, partials, fields, s);
  CNSF_CASE(0, 0) CNSF_CASE(0, 1) CNSF_CASE(0, 2)
  CNSF_CASE(1, 0) CNSF_CASE(1, 1) CNSF_CASE(1, 2)
  CNSF_CASE(2, 0) CNSF_CASE(2, 1) CNSF_CASE(2, 2)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_spectral(const Geom& g, double dx, double* fields, DiagPartial* partials, hipStream_t s) {
  const uint32_t dims[3] = {g.nx, g.ny, g.nz};
  const uint32_t strides[3] = {1u, g.nx, g.nxy};
  for (int a = 0; a < 3; ++a) {
    AxisGeom ag{};
    ag.n = dims[a];
    ag.stride = strides[a];
    ag.nlines = g.ncells / dims[a];
    uint32_t lg = 0;
    while ((1u << lg) < ag.n) ++lg;
    ag.log2n = ((1u << lg) == ag.n && ag.n >= 2) ? lg : 0;
    // LDS: 2 (FFT) or 4 (direct) complex rows per line plus the kernel, <= 64 KiB
    const uint32_t rows = ag.log2n ? 2u : 4u;
    uint32_t tl = (65536u - (ag.n + 2) * 8u) / (rows * ag.n * 16u);
    ag.lines_per_block = tl < 1 ? 1 : (tl > 16 ? 16 : tl);
    ag.axis = a;
    ag.last = (a == 2);
    ag.kscale = 2.0 * M_PI / ((double)ag.n * dx);
    const size_t lds = (size_t)rows * ag.lines_per_block * ag.n * sizeof(double2) + (size_t)(ag.n + 2) * sizeof(double);
    hipLaunchKernelGGL(k_spectral_axis, dim3(DIAG_BLOCKS), dim3(DB), lds, s, fields, g, ag, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_diag_final(DiagPartial* partials, int nparts, DiagPartial* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DB), 0, s, partials, nparts, out);
  return hipGetLastError();
}

}  // namespace cnsf
