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
#include <algorithm>
#include <cmath>

#include "cnsf_impl.h"
#include "diag_common.h"
#include "launch.h"

namespace cnsf {

constexpr int DB = 256;  // threads per diagnostics block
#ifndef CNSF_DERIV_PAIRS_X
// Line pairs per block of the derivative passes, and the unroll of their
// global loads and stores (512^3 FP32, HIP events, results bitwise equal):
// two pairs along x (more blocks per CU; the lines are contiguous anyway) and
// four along y and z (64-byte x-runs, three blocks per CU) take the nine
// passes and the readout from 17.9 to 15.1 ms; three pairs (48-byte runs) or
// nine to eleven (one block per CU) are slower.
#define CNSF_DERIV_PAIRS_X 2   // line pairs per block of the x-axis derivative pass (0: as many as fit)
#endif
#ifndef CNSF_DERIV_PAIRS_YZ
#define CNSF_DERIV_PAIRS_YZ 4  // line pairs per block of the y and z passes (0: as many as fit)
#endif
#ifndef CNSF_DERIV_LDS
#define CNSF_DERIV_LDS 65536   // LDS bytes a derivative-pass block may use
#endif
#ifndef CNSF_DERIV_UNROLL
#define CNSF_DERIV_UNROLL 4    // unroll of the derivative pass's global load and store loops
#endif
constexpr int kDerivUnroll = CNSF_DERIV_UNROLL;
#ifndef CNSF_DERIV_512
#define CNSF_DERIV_512 1       // 512-point lines take the register transform (k_deriv512)
#endif
#ifndef CNSF_SPEC_LINES_X
// Complex lines per block of the spectrum's axis passes, for the same reason
// as the derivative passes: 512^3, results bitwise equal, 28.3-29.1 ms with
// six lines everywhere, 25.4 ms with three along x and four along y and z.
#define CNSF_SPEC_LINES_X 3    // complex lines per block of the spectrum's x pass (0: as many as fit)
#endif
#ifndef CNSF_SPEC_LINES_YZ
#define CNSF_SPEC_LINES_YZ 4   // complex lines per block of its y and z passes (0: as many as fit)
#endif

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
    // the stored values are FP32 or 16-bit: gather them in FP32 (exact), sum in FP64
    float gf[NC][NV];
    gather<ST, BC, true, float>(pop, g, cd, n, parity, off, gf);
    cell_sums(gf, cd, phd, c, g.ncells, fields, acc);
    // the sensor decision as the FP32 update takes it
    float dQf[NC], Qf[NC];
    DevPrim Pf;
    float chi = 0.0f;
    cell_state(gf, cd, ph, dQf, Qf, Pf, &chi);
    acc.sensor += chi > 0.0f ? 1.0 : 0.0;
  }
  DiagPartial tot = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// The velocity alone, for the shell spectrum of a periodic lattice: only the
// 28 populations of rho and rho u are read (136 bytes per FP32 cell against
// the 392 + 32 of the full readout), and u = rho u / rho is formed in the
// full readout's arithmetic (FP64 sums of the stored values in slot order,
// then one reciprocal of rho).
template <int ST>
__global__ void __launch_bounds__(DB) k_velocity(const typename Store<ST>::T* __restrict__ pop, const Geom g,
                                                 const Codec cd, int parity, double* __restrict__ fields) {
  const uint32_t stride = gridDim.x * DB;
  for (uint32_t c = blockIdx.x * DB + threadIdx.x; c < g.ncells; c += stride) {
    const Nbr n = neighbours(c, g);
    uint32_t off[NV];
    stream_offsets<ST, 0>(g, n, parity, off);
    double Q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const __amdgpu_buffer_rsrc_t rs = component_rsrc<ST>(pop, g, k);
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        float v = buf_load<ST>(rs, off[i]);
        if (ST != 0) v *= cd.scale[k];
        sum += (double)v;
      }
      Q[k] = q_ref<double>(cd, k) + sum;
    }
    const double inv_rho = 1.0 / Q[0];
    fields[c] = Q[1] * inv_rho;
    fields[g.ncells + c] = Q[2] * inv_rho;
    fields[2 * (uint64_t)g.ncells + c] = Q[3] * inv_rho;
  }
}

// ------------------------------------------------------------------ spectral
// One derivative pass: d_a u_c for every line along axis a.
struct DerivAxis {
  uint32_t n;               // line length
  uint32_t stride;          // element stride along the line
  uint32_t nlines;
  uint32_t pairs_per_block; // line pairs held in LDS at once
  uint32_t log2n;           // 0 if n is not a power of two
  int axis;                 // 0 x, 1 y, 2 z
  int init;                 // store into the accumulator instead of adding
  int eps;                  // k_deriv512 only: 0 store the result; otherwise the pass completes
                            // its field and adds mu field^2 to the block's partial instead:
                            // 1 added to the partial's eps field, 2 the first such pass with
                            // whole partials (other fields neutral), 3 the first such pass
                            // into the eps fields only
  int eps_d;                // the completed field is div u (eps_d), else a vorticity component
  double sign;
  double kscale;            // 2 pi / (n dx)
};

__device__ inline uint32_t line_base(uint32_t l, int axis, const Geom& g) {
  if (axis == 0) return l * g.nx;                       // l = y + ny z
  if (axis == 1) return (l / g.nx) * g.nxy + (l % g.nx);  // l = x + nx z
  return l;                                             // l = x + nx y
}

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// Line groups per block, XCD-contiguous: the hardware deals blocks
// round-robin over the 8 XCDs, and gridDim.x is a multiple of 8, so XCD j
// (blocks b = j mod 8) walks the j-th eighth of the groups in order.  In the
// y and z passes neighbouring groups read neighbouring x, i.e. the same cache
// lines, which then stay in one L2.
struct GroupRange {
  uint32_t begin, end, step;
};
__device__ inline GroupRange xcd_groups(uint32_t groups) {
  const uint32_t x = blockIdx.x & 7u, per = (groups + 7u) / 8u;
  GroupRange r;
  r.begin = x * per + (blockIdx.x >> 3);
  r.end = min(groups, (x + 1u) * per);
  r.step = gridDim.x >> 3;
  return r;
}

// LDS layout of a line: element p at p + p/8 (one 16-byte pad per 128 bytes),
// so the power-of-two strides of the bit-reversed loads and of the butterflies
// spread over all banks.
__device__ inline uint32_t lds_idx(uint32_t p) { return p + (p >> 3); }
__host__ __device__ inline uint32_t lds_line(uint32_t n) { return n + (n >> 3); }

// Per-stage twiddles: stage h (a power of two) keeps exp(-i pi m / h), m < h,
// at tw[h - 1 + m]; n - 1 entries, filled once per block.
__device__ inline void fill_twiddles(double2* tw, uint32_t n) {
  for (uint32_t q = threadIdx.x; q + 1 < n; q += blockDim.x) {
    const uint32_t h = 1u << (31 - __clz(q + 1)), m = q + 1 - h;
    double s, c;
    sincospi(-(double)m / (double)h, &s, &c);
    tw[q] = make_double2(c, s);
  }
}

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 conj2(double2 w) { return make_double2(w.x, -w.y); }

// In-place transform of `cnt` lines of length n = 2^log2n held in LDS (line
// stride lds_line(n)): forward decimation in time from bit-reversed input, or
// inverse decimation in frequency from natural input (output bit-reversed).
// Pairs of radix-2 stages are fused into one radix-4 step (four values per
// thread, one LDS round trip and one barrier for two stages); the arithmetic
// is that of the two stages in their order, so the result is the radix-2
// transform's bit for bit.  An odd stage count ends with one radix-2 stage.
__device__ inline void fft_dit(double2* buf, uint32_t n, uint32_t log2n, uint32_t cnt, const double2* tw) {
  const uint32_t np = lds_line(n);
  uint32_t s = 0;
  if (log2n >= 2) {
    const uint32_t lq = log2n - 2, qmask = (n >> 2) - 1u, totq = cnt << lq;
    for (; s + 1 < log2n; s += 2) {
      const uint32_t h = 1u << s;
      for (uint32_t t = threadIdx.x; t < totq; t += blockDim.x) {
        const uint32_t q = t & qmask;
        const uint32_t m = q & (h - 1u), j = ((q >> s) << (s + 2)) + m;
        double2* L = buf + (t >> lq) * np;
        const uint32_t i0 = lds_idx(j), i1 = lds_idx(j + h), i2 = lds_idx(j + 2 * h), i3 = lds_idx(j + 3 * h);
        const double2 a0 = L[i0], a1 = L[i1], a2 = L[i2], a3 = L[i3];
        const double2 w1 = tw[h - 1 + m];
        const double2 t1 = cmul(w1, a1), t3 = cmul(w1, a3);
        const double2 b0 = cadd(a0, t1), b1 = csub(a0, t1), b2 = cadd(a2, t3), b3 = csub(a2, t3);
        const double2 u2 = cmul(tw[2 * h - 1 + m], b2), u3 = cmul(tw[2 * h - 1 + m + h], b3);
        L[i0] = cadd(b0, u2);
        L[i2] = csub(b0, u2);
        L[i1] = cadd(b1, u3);
        L[i3] = csub(b1, u3);
      }
      __syncthreads();
    }
  }
  if (s < log2n) {
    const uint32_t lh = log2n - 1, hmask = (n >> 1) - 1u, total = cnt << lh, h = 1u << s;
    for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) {
      const uint32_t b = t & hmask;
      const uint32_t m = b & (h - 1u), j = ((b >> s) << (s + 1)) + m;
      double2* L = buf + (t >> lh) * np;
      const uint32_t i0 = lds_idx(j), i1 = lds_idx(j + h);
      const double2 x0 = L[i0], x1 = cmul(tw[h - 1 + m], L[i1]);
      L[i0] = cadd(x0, x1);
      L[i1] = csub(x0, x1);
    }
    __syncthreads();
  }
}

__device__ inline void fft_dif_inv(double2* buf, uint32_t n, uint32_t log2n, uint32_t cnt, const double2* tw) {
  const uint32_t np = lds_line(n);
  int s = (int)log2n - 1;
  if (log2n >= 2) {
    const uint32_t lq = log2n - 2, qmask = (n >> 2) - 1u, totq = cnt << lq;
    for (; s >= 1; s -= 2) {
      const uint32_t h = 1u << s, hh = h >> 1;
      for (uint32_t t = threadIdx.x; t < totq; t += blockDim.x) {
        const uint32_t q = t & qmask;
        const uint32_t m = q & (hh - 1u), j = ((q >> (s - 1)) << (s + 1)) + m;
        double2* L = buf + (t >> lq) * np;
        const uint32_t i0 = lds_idx(j), i1 = lds_idx(j + hh), i2 = lds_idx(j + 2 * hh), i3 = lds_idx(j + 3 * hh);
        const double2 a0 = L[i0], a1 = L[i1], a2 = L[i2], a3 = L[i3];
        const double2 c0 = cadd(a0, a2), c2 = cmul(csub(a0, a2), conj2(tw[h - 1 + m]));
        const double2 c1 = cadd(a1, a3), c3 = cmul(csub(a1, a3), conj2(tw[h - 1 + m + hh]));
        const double2 w = conj2(tw[hh - 1 + m]);
        L[i0] = cadd(c0, c1);
        L[i1] = cmul(csub(c0, c1), w);
        L[i2] = cadd(c2, c3);
        L[i3] = cmul(csub(c2, c3), w);
      }
      __syncthreads();
    }
  }
  if (s == 0) {
    const uint32_t lh = log2n - 1, total = cnt << lh;
    const double2 w = conj2(tw[0]);
    for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) {
      const uint32_t j = (t & ((n >> 1) - 1u)) << 1;
      double2* L = buf + (t >> lh) * np;
      const uint32_t i0 = lds_idx(j), i1 = lds_idx(j + 1);
      const double2 x0 = L[i0], x1 = L[i1];
      L[i0] = cadd(x0, x1);
      L[i1] = cmul(csub(x0, x1), w);
    }
    __syncthreads();
  }
}

// Spectral derivative along axis a of one velocity component, two adjacent
// lines per complex transform: z = u_c(l) + i u_c(l+1).  The derivative
// (multiply by i kappa, Nyquist mode to zero) is a real-linear map, so the
// real and imaginary parts of D z are the derivatives of the two lines.  The
// result times `sign` is stored into (init) or added to the accumulator, one
// of div u, omega_x, omega_y, omega_z.  Powers of two use the LDS transform,
// other lengths the spectral-derivative kernel as a direct sum.
__global__ void __launch_bounds__(DB) k_deriv_axis(const double* __restrict__ uc, double* __restrict__ acc, const Geom g,
                                                   const DerivAxis da) {
  extern __shared__ double2 lds[];
  const uint32_t n = da.n, TP = da.pairs_per_block, np = lds_line(n);
  const bool pow2 = da.log2n != 0;
  double2* A = lds;
  double2* Aout = pow2 ? A : lds + TP * np;
  double2* tw = lds + TP * np;                      // power of two
  double* Dk = (double*)(lds + 2 * TP * np);        // direct
  if (pow2) {
    fill_twiddles(tw, n);
  } else {
    // D[m] = -(2/n) sum_{k=1}^{K} kappa_k sin(2 pi k m / n), Nyquist excluded
    const uint32_t K = (n % 2) ? (n - 1) / 2 : n / 2 - 1;
    for (uint32_t m = threadIdx.x; m < n; m += blockDim.x) {
      double sacc = 0.0;
      for (uint32_t k = 1; k <= K; ++k) sacc += (double)k * sinpi(2.0 * (double)((uint64_t)k * m % n) / (double)n);
      Dk[m] = -2.0 / (double)n * da.kscale * sacc;
    }
  }
  const uint32_t npairs = (da.nlines + 1) / 2;
  const GroupRange gr = xcd_groups((npairs + TP - 1) / TP);
  for (uint32_t grp = gr.begin; grp < gr.end; grp += gr.step) {
    const uint32_t p0 = grp * TP;
    const uint32_t cnt = min(TP, npairs - p0);
    __syncthreads();
    // load (bit-reversed positions for the decimation-in-time transform);
    // along y and z, consecutive threads take consecutive line pairs
#pragma unroll kDerivUnroll
    for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
      uint32_t pr, j;
      if (da.axis == 0) { pr = e / n; j = e % n; }
      else { pr = e % cnt; j = e / cnt; }
      const uint32_t l0 = 2 * (p0 + pr);
      const double x0 = uc[line_base(l0, da.axis, g) + j * da.stride];
      const double x1 = l0 + 1 < da.nlines ? uc[line_base(l0 + 1, da.axis, g) + j * da.stride] : 0.0;
      const uint32_t pos = pow2 ? (__brev(j) >> (32 - da.log2n)) : j;
      A[pr * np + lds_idx(pos)] = make_double2(x0, x1);
    }
    __syncthreads();
    if (pow2) {
      fft_dit(A, n, da.log2n, cnt, tw);
      // multiply by i kappa_j (Nyquist to zero) and 1/n for the inverse
      for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
        const uint32_t j = e & (n - 1u), q = (e >> da.log2n) * np + lds_idx(j);
        double kj = (j < n / 2) ? (double)j : (j == n / 2 ? 0.0 : (double)j - (double)n);
        kj *= da.kscale / (double)n;
        const double2 x = A[q];
        A[q] = make_double2(-kj * x.y, kj * x.x);
      }
      __syncthreads();
      fft_dif_inv(A, n, da.log2n, cnt, tw);   // output in bit-reversed positions
    } else {
      // direct: d_j = sum_m D[m] z_{(j - m) mod n}
      for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
        const uint32_t pr = e / n, j = e % n;
        double dr = 0.0, di = 0.0;
        for (uint32_t m = 0; m < n; ++m) {
          const double2 z = A[pr * np + lds_idx((j + n - m) % n)];
          const double d = Dk[m];
          dr += d * z.x;
          di += d * z.y;
        }
        Aout[pr * np + lds_idx(j)] = make_double2(dr, di);
      }
      __syncthreads();
    }
#pragma unroll kDerivUnroll
    for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
      uint32_t pr, j;
      if (da.axis == 0) { pr = e / n; j = e % n; }
      else { pr = e % cnt; j = e / cnt; }
      const uint32_t l0 = 2 * (p0 + pr);
      const uint32_t pos = pow2 ? (__brev(j) >> (32 - da.log2n)) : j;
      const double2 r = Aout[pr * np + lds_idx(pos)];
      const uint32_t a0 = line_base(l0, da.axis, g) + j * da.stride;
      acc[a0] = da.init ? da.sign * r.x : acc[a0] + da.sign * r.x;
      if (l0 + 1 < da.nlines) {
        const uint32_t a1 = line_base(l0 + 1, da.axis, g) + j * da.stride;
        acc[a1] = da.init ? da.sign * r.y : acc[a1] + da.sign * r.y;
      }
    }
  }
}

// ------------------------------------------------------------------ 512-point lines
// Lines of 512 points (the 512^3 box) take a transform held in registers: one
// wavefront per line pair, eight values per lane, three radix-8 steps with
// two exchanges through the wave's own LDS slice (512 = 8 x 8 x 8), forward
// from natural order to digit-reversed order and the inverse back.  With
// j = t + 64 m (t the lane) and k = k2 + 8 k1 + 64 k0:
//   step 1: lane t sums over m (radix 8), twiddle w^(t k2);
//   step 2: lane (t mod 8, k2) sums over t div 8, twiddle w^(8 (t mod 8) k1);
//   step 3: lane (k1, k2) sums over t mod 8 and holds Z[k2 + 8 k1 + 64 k0].
// The inverse runs the same steps backwards with conjugate twiddles.
constexpr uint32_t L512_ROW = 65;                 // exchange row: 64 values and one pad
constexpr uint32_t L512_WAVE = 8 * L512_ROW;      // complex values per wave slice

__device__ inline double2 mul_j(double2 a, int S) {   // a * exp(S i pi / 2)
  return S < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// V[k] = sum_m v[m] exp(S 2 pi i m k / 8), natural order in and out.
template <int S>
__device__ inline void dft8(double2 (&v)[8]) {
  constexpr double c = 0.70710678118654752440;
  double2 e[4], o[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {                    // the two length-4 transforms, even and odd inputs
    const double2 a0 = v[h], a1 = v[h + 2], a2 = v[h + 4], a3 = v[h + 6];
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_j(csub(a1, a3), S);
    double2* r = h ? o : e;
    r[0] = cadd(t0, t2);
    r[2] = csub(t0, t2);
    r[1] = cadd(t1, t3);
    r[3] = csub(t1, t3);
  }
  // W^k o[k], W = exp(S i pi / 4)
  const double2 w1 = make_double2(c, S * c), w3 = make_double2(-c, S * c);
  const double2 p0 = o[0], p1 = cmul(w1, o[1]), p2 = mul_j(o[2], S), p3 = cmul(w3, o[3]);
  v[0] = cadd(e[0], p0);
  v[4] = csub(e[0], p0);
  v[1] = cadd(e[1], p1);
  v[5] = csub(e[1], p1);
  v[2] = cadd(e[2], p2);
  v[6] = csub(e[2], p2);
  v[3] = cadd(e[3], p3);
  v[7] = csub(e[3], p3);
}

// Order the wave's LDS accesses: writes of every lane before any later read.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward transform: lane t holds z[t + 64 m] in v[m]; on return lane
// (k1 + 8 k2) holds Z[k2 + 8 k1 + 64 k0] in v[k0].  X is the wave's LDS slice,
// tw[r] = exp(-2 pi i r / 512).
__device__ inline void fft512_fwd(double2 (&v)[8], double2* X, const double2* tw, uint32_t lane) {
  dft8<-1>(v);
#pragma unroll
  for (int k2 = 1; k2 < 8; ++k2) v[k2] = cmul(v[k2], tw[(lane * k2) & 511u]);
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) X[k2 * L512_ROW + lane] = v[k2];
  wave_lds_sync();
  const uint32_t t1 = lane & 7u, k2 = lane >> 3;
#pragma unroll
  for (int t2 = 0; t2 < 8; ++t2) v[t2] = X[k2 * L512_ROW + t1 + 8 * t2];
  wave_lds_sync();
  dft8<-1>(v);
#pragma unroll
  for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], tw[(8u * t1 * k1) & 511u]);
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) X[k2 * L512_ROW + 8 * k1 + t1] = v[k1];
  wave_lds_sync();
  const uint32_t k1 = lane & 7u;
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = X[k2 * L512_ROW + 8 * k1 + u];
  wave_lds_sync();
  dft8<-1>(v);
}

// Inverse (unnormalised): lane (k1 + 8 k2) holds Z[k2 + 8 k1 + 64 k0] in v[k0];
// on return lane t holds z[t + 64 m] in v[m].
__device__ inline void fft512_inv(double2 (&v)[8], double2* X, const double2* tw, uint32_t lane) {
  dft8<1>(v);                                       // over k0: index t1
  const uint32_t k1 = lane & 7u, k2 = lane >> 3;
#pragma unroll
  for (int t1 = 0; t1 < 8; ++t1) X[k2 * L512_ROW + 8 * k1 + t1] = v[t1];
  wave_lds_sync();
  const uint32_t t1 = lane & 7u;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) v[kk] = cmul(X[k2 * L512_ROW + 8 * kk + t1], conj2(tw[(8u * t1 * kk) & 511u]));
  wave_lds_sync();
  dft8<1>(v);                                       // over k1: index t2
#pragma unroll
  for (int t2 = 0; t2 < 8; ++t2) X[k2 * L512_ROW + t1 + 8 * t2] = v[t2];
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = cmul(X[q * L512_ROW + lane], conj2(tw[(lane * q) & 511u]));
  wave_lds_sync();
  dft8<1>(v);                                       // over k2: index m
}

// Spectral derivative of 512-point lines (any axis), as k_deriv_axis: two
// adjacent lines per complex transform, the result times `sign` stored into
// or added to the accumulator.  A block of eight wavefronts takes a group of
// eight line pairs (sixteen consecutive lines), one wavefront per pair, groups
// in XCD-contiguous order.  Along x a lane reads its eight points straight
// from memory (each load covers 64 consecutive points).  Along y and z the
// sixteen lines are neighbours in x, so the block reads and writes them
// through LDS in rows of sixteen consecutive x (whole 128-byte lines),
// instead of 64 separate rows per load.
//
// A pass that completes a field (the last of its derivative terms) can also
// reduce its Eq. (7) sum: with da.eps set it reads mu at each point, adds
// mu field^2 to the block's partial (eps_s for a vorticity component, eps_d
// for div u), and does not store the field, which nothing reads afterwards.
constexpr int W512 = 8;                            // wavefronts per block of the 512-point kernels
template <bool EPS>
__global__ void __launch_bounds__(64 * W512) k_deriv512(const double* __restrict__ uc, double* __restrict__ acc,
                                                        const Geom g, const DerivAxis da,
                                                        const double* __restrict__ fields,
                                                        DiagPartial* __restrict__ partials) {
  __shared__ double2 tw[512];
  __shared__ double2 xch[W512 * L512_WAVE];
  double* S = (double*)xch;                        // y, z: staging rows, S[line * 513 + j]
  constexpr uint32_t SROW = 513;
  constexpr uint32_t GL = 2 * W512;                // lines per group
  for (uint32_t r = threadIdx.x; r < 512; r += blockDim.x) {
    double sn, cs;
    sincospi(-(double)r / 256.0, &sn, &cs);
    tw[r] = make_double2(cs, sn);
  }
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  double2* X = xch + wave * L512_WAVE;
  const GroupRange gr = xcd_groups((da.nlines + GL - 1) / GL);
  const double kf = da.kscale / 512.0;
  double esum = 0.0;                               // EPS: sum of mu field^2 over this thread's points
  const uint32_t kb = (lane >> 3) + 8u * (lane & 7u);   // k = kb + 64 k0 after the forward transform
  // y and z staging: thread t serves line sn = t mod GL of its group at the
  // points j0 + JSTEP q, q < PER
  constexpr uint32_t JSTEP = 64 * W512 / GL, PER = 512 / JSTEP;
  static_assert((64 * W512) % GL == 0 && 512 % JSTEP == 0, "staging layout");
  const uint32_t sn = threadIdx.x % GL, j0 = threadIdx.x / GL;
  const uint64_t qstep = (uint64_t)JSTEP * da.stride;   // elements between a thread's points
  double ld[PER];
  for (uint32_t grp = gr.begin; grp < gr.end; grp += gr.step) {
    const uint32_t lfirst = GL * grp;                  // first line of the group
    const uint32_t nl = min(GL, da.nlines - lfirst);   // lines in the group
    const uint32_t l0 = lfirst + 2 * wave;             // this wave's pair
    const bool live = 2 * wave < nl, two = 2 * wave + 1 < nl;
    const bool sl = sn < nl;                           // this thread's staging line exists
    const uint32_t toff = sl ? line_base(lfirst + sn, da.axis, g) + j0 * da.stride : 0u;
    double2 v[8];
    __syncthreads();
    if (da.axis == 0) {
      if (live) {
        const uint32_t b0 = line_base(l0, 0, g), b1 = two ? line_base(l0 + 1, 0, g) : b0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t j = lane + 64u * m;
          v[m] = make_double2(uc[b0 + j], two ? uc[b1 + j] : 0.0);
        }
      }
    } else {
      // Thread t always serves line t mod GL at points j0 + JSTEP q: one
      // per-thread offset and a block-uniform step, so all PER loads are in
      // flight before the first LDS write.
#pragma unroll
      for (int q = 0; q < PER; ++q) ld[q] = sl ? (uc + q * qstep)[toff] : 0.0;
#pragma unroll
      for (int q = 0; q < PER; ++q) S[sn * SROW + j0 + JSTEP * q] = ld[q];
      __syncthreads();
      if (live) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t j = lane + 64u * m;
          v[m] = make_double2(S[(2 * wave) * SROW + j], two ? S[(2 * wave + 1) * SROW + j] : 0.0);
        }
      }
      __syncthreads();                                 // the exchanges below reuse S
    }
    if (live) {
      fft512_fwd(v, X, tw, lane);
      // times i kappa / 512, the Nyquist mode to zero
#pragma unroll
      for (int k0 = 0; k0 < 8; ++k0) {
        const uint32_t k = kb + 64u * k0;
        const double ks = k < 256u ? (double)k : (k == 256u ? 0.0 : (double)k - 512.0);
        const double f = ks * kf;
        v[k0] = make_double2(-f * v[k0].y, f * v[k0].x);
      }
      fft512_inv(v, X, tw, lane);
    }
    if (da.axis == 0) {
      if (live) {
        const uint32_t b0 = line_base(l0, 0, g), b1 = two ? line_base(l0 + 1, 0, g) : b0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t j = lane + 64u * m;
          acc[b0 + j] = da.init ? da.sign * v[m].x : acc[b0 + j] + da.sign * v[m].x;
          if (two) acc[b1 + j] = da.init ? da.sign * v[m].y : acc[b1 + j] + da.sign * v[m].y;
        }
      }
    } else {
      __syncthreads();                                 // every wave is done with its exchanges
      if (live) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t j = lane + 64u * m;
          S[(2 * wave) * SROW + j] = v[m].x;
          if (two) S[(2 * wave + 1) * SROW + j] = v[m].y;
        }
      }
      __syncthreads();
      if constexpr (EPS) {
        // the completed field at each point, mu times its square summed
        const double* mu = fields + 3 * (uint64_t)g.ncells;
#pragma unroll
        for (int q0 = 0; q0 < (int)PER; q0 += 8) {
          double av[8], mv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const uint64_t o = (uint64_t)(q0 + q) * qstep;
            av[q] = (sl && !da.init) ? (acc + o)[toff] : 0.0;
            mv[q] = sl ? (mu + o)[toff] : 0.0;
          }
          if (sl) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const double d = av[q] + da.sign * S[sn * SROW + j0 + JSTEP * (q0 + q)];
              esum += mv[q] * d * d;
            }
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) ld[q] = (sl && !da.init) ? (acc + q * qstep)[toff] : 0.0;
        if (sl) {
#pragma unroll
          for (int q = 0; q < PER; ++q) (acc + q * qstep)[toff] = ld[q] + da.sign * S[sn * SROW + j0 + JSTEP * q];
        }
      }
    }
  }
  if constexpr (EPS) {
    // block sum in a fixed order: wave shuffles, then the waves in index order
    __shared__ double red[W512];
    esum = wave_sum(esum);
    __syncthreads();
    if (lane == 0) red[wave] = esum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = red[0];
      for (int w = 1; w < W512; ++w) t += red[w];
      DiagPartial& P = partials[blockIdx.x];
      if (da.eps == 2) {
        DiagPartial p;
        part_zero(p);
        (da.eps_d ? p.eps_d : p.eps_s) = t;
        P = p;
      } else if (da.eps == 3) {
        P.eps_s = da.eps_d ? 0.0 : t;
        P.eps_d = da.eps_d ? t : 0.0;
      } else {
        (da.eps_d ? P.eps_d : P.eps_s) += t;
      }
    }
  }
}

// eps sums: sum of mu |omega|^2 and mu (div u)^2 over the cells, per block,
// into the eps fields of the block's partial (full: a whole partial, the
// other fields neutral).
__global__ void __launch_bounds__(DB) k_eps_sums(const double* __restrict__ fields, const Geom g,
                                                 DiagPartial* __restrict__ partials, int full) {
  const uint64_t N = g.ncells;
  const double* mu = fields + 3 * N;
  const double* divf = fields + 4 * N;
  const double* wx = fields + 5 * N;
  const double* wy = fields + 6 * N;
  const double* wz = fields + 7 * N;
  DiagPartial acc;
  part_zero(acc);
  for (uint32_t c = blockIdx.x * DB + threadIdx.x; c < g.ncells; c += gridDim.x * DB) {
    const double m = mu[c], d = divf[c], x = wx[c], y = wy[c], z = wz[c];
    acc.eps_s += m * (x * x + y * y + z * z);
    acc.eps_d += m * d * d;
  }
  DiagPartial tot = block_reduce(acc);
  if (threadIdx.x == 0) {
    if (full) {
      partials[blockIdx.x] = tot;
    } else {
      partials[blockIdx.x].eps_s = tot.eps_s;
      partials[blockIdx.x].eps_d = tot.eps_d;
    }
  }
}

// ------------------------------------------------------------------ shell spectrum
// Forward transform along one axis of the velocity component being processed:
// mode 0 reads the real field and writes complex, mode 1 transforms the complex
// workspace in place, mode 2 transforms and stores (or adds) |X|^2 * escale
// into the energy field.  Powers of two use the LDS radix-2 transform; other
// lengths a direct sum.
struct SpecAxis {
  uint32_t n, stride, nlines, lines_per_block, log2n;
  int axis;
  int mode;
  int accumulate;
  double escale;
};

__global__ void __launch_bounds__(DB) k_spectrum_axis(const double* __restrict__ real_in, double2* __restrict__ data,
                                                      double* __restrict__ energy, const Geom g, const SpecAxis sa) {
  extern __shared__ double2 lds[];
  const uint32_t n = sa.n, TL = sa.lines_per_block;
  const bool pow2 = sa.log2n != 0;
  const uint32_t np = lds_line(n);
  double2* A = lds;
  double2* Aout = pow2 ? A : lds + TL * np;
  double2* tw = lds + TL * np;                           // power of two
  if (pow2) fill_twiddles(tw, n);
  const GroupRange gr = xcd_groups((sa.nlines + TL - 1) / TL);
  for (uint32_t grp = gr.begin; grp < gr.end; grp += gr.step) {
    const uint32_t l0 = grp * TL;
    const uint32_t cnt = min(TL, sa.nlines - l0);
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
      uint32_t line, j;
      if (sa.axis == 0) { line = e / n; j = e % n; }
      else { line = e % cnt; j = e / cnt; }
      const uint32_t addr = line_base(l0 + line, sa.axis, g) + j * sa.stride;
      const uint32_t pos = pow2 ? (__brev(j) >> (32 - sa.log2n)) : j;
      A[line * np + lds_idx(pos)] = sa.mode == 0 ? make_double2(real_in[addr], 0.0) : data[addr];
    }
    __syncthreads();
    if (pow2) {
      fft_dit(A, n, sa.log2n, cnt, tw);   // natural-order output
    } else {
      for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
        const uint32_t line = e / n, k = e % n;
        double re = 0.0, im = 0.0;
        for (uint32_t m = 0; m < n; ++m) {
          double sn, cs;
          sincospi(-2.0 * (double)((uint64_t)k * m % n) / (double)n, &sn, &cs);
          const double2 x = A[line * np + lds_idx(m)];
          re += x.x * cs - x.y * sn;
          im += x.x * sn + x.y * cs;
        }
        Aout[line * np + lds_idx(k)] = make_double2(re, im);
      }
      __syncthreads();
    }
    for (uint32_t e = threadIdx.x; e < cnt * n; e += blockDim.x) {
      uint32_t line, j;
      if (sa.axis == 0) { line = e / n; j = e % n; }
      else { line = e % cnt; j = e / cnt; }
      const uint32_t addr = line_base(l0 + line, sa.axis, g) + j * sa.stride;
      const double2 X = Aout[line * np + lds_idx(j)];
      if (sa.mode == 2) {
        const double v = (X.x * X.x + X.y * X.y) * sa.escale;
        energy[addr] = sa.accumulate ? energy[addr] + v : v;
      } else {
        data[addr] = X;
      }
    }
  }
}

// Forward transform of 512-point lines for the shell spectrum (as
// k_spectrum_axis, same modes): one wavefront per complex line, eight
// consecutive lines per block, the register transform of the derivative
// passes, results in natural order.  Along y and z the eight lines are
// neighbours in x and go through LDS in rows of eight (128-byte runs).
__global__ void __launch_bounds__(64 * W512) k_spectrum512(const double* __restrict__ real_in,
                                                           double2* __restrict__ data, double* __restrict__ energy,
                                                           const Geom g, const SpecAxis sa) {
  __shared__ double2 tw[512];
  __shared__ double2 xch[W512 * L512_WAVE];
  double2* S = xch;                                // y, z: staging rows, S[line * 513 + k]
  constexpr uint32_t SROW = 513;
  for (uint32_t r = threadIdx.x; r < 512; r += blockDim.x) {
    double sn, cs;
    sincospi(-(double)r / 256.0, &sn, &cs);
    tw[r] = make_double2(cs, sn);
  }
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  double2* X = xch + wave * L512_WAVE;
  constexpr uint32_t GL = W512;                    // lines per group
  const GroupRange gr = xcd_groups((sa.nlines + GL - 1) / GL);
  const uint32_t kb = (lane >> 3) + 8u * (lane & 7u);
  // y and z staging: thread t serves line sn = t mod GL of its group at the
  // points j0 + JSTEP q, q < PER (one per-thread offset, a block-uniform step)
  constexpr uint32_t JSTEP = 64 * W512 / GL, PER = 512 / JSTEP;
  static_assert((64 * W512) % GL == 0 && 512 % JSTEP == 0, "staging layout");
  const uint32_t sn = threadIdx.x % GL, j0 = threadIdx.x / GL;
  const uint64_t qstep = (uint64_t)JSTEP * sa.stride;
  for (uint32_t grp = gr.begin; grp < gr.end; grp += gr.step) {
    const uint32_t lfirst = GL * grp, nl = min(GL, sa.nlines - lfirst);
    const uint32_t line = lfirst + wave;
    const bool live = wave < nl;
    const bool sl = sn < nl;
    const uint32_t toff = sl ? line_base(lfirst + sn, sa.axis, g) + j0 * sa.stride : 0u;
    double2 v[8];
    __syncthreads();
    if (sa.axis == 0) {
      if (live) {
        const uint32_t b = line_base(line, 0, g);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t addr = b + lane + 64u * m;
          v[m] = sa.mode == 0 ? make_double2(real_in[addr], 0.0) : data[addr];
        }
      }
    } else {
      // all of the thread's loads in flight before the LDS writes
      double2 ld[PER];
      if (sa.mode == 0) {
#pragma unroll
        for (int q = 0; q < (int)PER; ++q) ld[q] = make_double2(sl ? (real_in + q * qstep)[toff] : 0.0, 0.0);
      } else {
#pragma unroll
        for (int q = 0; q < (int)PER; ++q) ld[q] = sl ? (data + q * qstep)[toff] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < (int)PER; ++q) S[sn * SROW + j0 + JSTEP * q] = ld[q];
      __syncthreads();
      if (live) {
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = S[wave * SROW + lane + 64u * m];
      }
      __syncthreads();                                 // the exchanges below reuse S
    }
    if (live) fft512_fwd(v, X, tw, lane);
    if (sa.axis == 0) {
      if (live) {
        const uint32_t b = line_base(line, 0, g);
#pragma unroll
        for (int k0 = 0; k0 < 8; ++k0) {
          const uint32_t addr = b + kb + 64u * k0;
          if (sa.mode == 2) {
            const double e = (v[k0].x * v[k0].x + v[k0].y * v[k0].y) * sa.escale;
            energy[addr] = sa.accumulate ? energy[addr] + e : e;
          } else {
            data[addr] = v[k0];
          }
        }
      }
    } else {
      __syncthreads();
      if (live) {
#pragma unroll
        for (int k0 = 0; k0 < 8; ++k0) S[wave * SROW + kb + 64u * k0] = v[k0];
      }
      __syncthreads();
      if (sa.mode == 2) {
        double ev[PER];
#pragma unroll
        for (int q = 0; q < (int)PER; ++q) ev[q] = (sl && sa.accumulate) ? (energy + q * qstep)[toff] : 0.0;
        if (sl) {
#pragma unroll
          for (int q = 0; q < (int)PER; ++q) {
            const double2 Xv = S[sn * SROW + j0 + JSTEP * q];
            (energy + q * qstep)[toff] = ev[q] + (Xv.x * Xv.x + Xv.y * Xv.y) * sa.escale;
          }
        }
      } else if (sl) {
#pragma unroll
        for (int q = 0; q < (int)PER; ++q) (data + q * qstep)[toff] = S[sn * SROW + j0 + JSTEP * q];
      }
    }
  }
}

// Integer wavenumber of DFT index j on an axis of n points.
__device__ inline int64_t wavenumber(uint32_t j, uint32_t n) { return j < (n + 1) / 2 ? (int64_t)j : (int64_t)j - n; }

// Shell sums of one kappa_z plane per block, in a fixed order.  Along a row of
// fixed (kappa_y, kappa_z) the shell nint(|kappa|) never decreases with
// |kappa_x|, so a wave takes 64 consecutive |kappa_x| (both signs together),
// sums each run of equal shells with a segmented scan, and adds the run totals
// to its own LDS histogram (shells within one chunk are distinct).  Wave w
// takes rows w, w + 4, ...; the block adds its four histograms in order.
__global__ void __launch_bounds__(DB) k_shell_partials(const double* __restrict__ energy, uint32_t n, uint32_t nshells,
                                                       double* __restrict__ partial) {
  extern __shared__ double hist[];   // 4 x nshells
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  for (uint32_t s = threadIdx.x; s < 4 * nshells; s += blockDim.x) hist[s] = 0.0;
  __syncthreads();
  const uint32_t jz = blockIdx.x;
  const int64_t mz = wavenumber(jz, n);
  const uint32_t tmax = n / 2;      // largest |kappa_x|
  double* h = hist + wave * nshells;
  for (uint32_t jy = wave; jy < n; jy += 4) {
    const int64_t my = wavenumber(jy, n);
    const int64_t c2 = my * my + mz * mz;
    const double* row = energy + ((uint64_t)jz * n + jy) * n;
    for (uint32_t t0 = 0; t0 <= tmax; t0 += 64) {
      const uint32_t t = t0 + lane;
      const bool valid = t <= tmax;
      int key = 0x7fffffff;
      double val = 0.0;
      if (valid) {
        key = (int)floor(sqrt((double)((int64_t)t * t + c2)) + 0.5);
        val = row[t];
        if (t != 0 && n - t != t) val += row[n - t];
      }
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const double ov = __shfl_up(val, d, 64);
        const int ok = __shfl_up(key, d, 64);
        if ((int)lane >= d && ok == key) val += ov;
      }
      const int next = __shfl_down(key, 1, 64);
      if (valid && (lane == 63 || next != key)) h[key] += val;
    }
  }
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < nshells; s += blockDim.x)
    partial[(uint64_t)jz * nshells + s] = ((hist[s] + hist[nshells + s]) + hist[2 * nshells + s]) + hist[3 * nshells + s];
}

// E[k] = sum over planes of the partial shell sums, planes in order; zero for
// k >= nshells up to nout.
__global__ void k_shell_final(const double* __restrict__ partial, uint32_t nplanes, uint32_t nshells, uint32_t nout,
                              double* __restrict__ E) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nout) return;
  double acc = 0.0;
  if (k < nshells)
    for (uint32_t p = 0; p < nplanes; ++p) acc += partial[(uint64_t)p * nshells + k];
  E[k] = acc;
}

// Sums of consecutive chunks of partials, one block per chunk, in a fixed order.
__global__ void k_diag_chunks(const DiagPartial* __restrict__ partials, int nparts, int chunk,
                              DiagPartial* __restrict__ out) {
  DiagPartial acc;
  part_zero(acc);
  const int lo = blockIdx.x * chunk, hi = min(nparts, lo + chunk);
  for (int i = lo + (int)threadIdx.x; i < hi; i += DB) part_add(acc, partials[i]);
  DiagPartial tot = block_reduce(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

__global__ void k_diag_final(const DiagPartial* __restrict__ partials, int nparts, DiagPartial* __restrict__ out) {
  DiagPartial acc;
  part_zero(acc);
  for (int i = threadIdx.x; i < nparts; i += DB) part_add(acc, partials[i]);
  DiagPartial tot = block_reduce(acc);
  if (threadIdx.x == 0) *out = tot;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_velocity(int storage, const void* pop, const Geom& g, const Codec& cd, int parity, double* fields,
                           hipStream_t s) {
  if (g.bc_x != 0) return hipErrorInvalidValue;
#define CNSF_CASE(ST)                                                                                              \
  if (storage == ST) {                                                                                             \
    hipLaunchKernelGGL((k_velocity<ST>), dim3(DIAG_BLOCKS), dim3(DB), 0, s, (const typename Store<ST>::T*)pop, g, \
                       cd, parity, fields);                                                                       \
    return hipGetLastError();                                                                                      \
  }
  CNSF_CASE(0) CNSF_CASE(1) CNSF_CASE(2)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

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
  CNSF_CASE(0, 0) CNSF_CASE(0, 1) CNSF_CASE(0, 2) CNSF_CASE(0, 3)
  CNSF_CASE(1, 0) CNSF_CASE(1, 1) CNSF_CASE(1, 2) CNSF_CASE(1, 3)
  CNSF_CASE(2, 0) CNSF_CASE(2, 1) CNSF_CASE(2, 2) CNSF_CASE(2, 3)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

// Nine derivative passes d_a u_c into div u = sum_a d_a u_a and
// omega_b = eps_{b a c} d_a u_c, then the eps sums.  The first pass into each
// accumulator stores, the later ones add.
hipError_t launch_spectral(const Geom& g, double dx, double* fields, DiagPartial* partials, bool full,
                           hipStream_t s) {
  const uint32_t dims[3] = {g.nx, g.ny, g.nz};
  const uint32_t strides[3] = {1u, g.nx, g.nxy};
  const uint64_t N = g.ncells;
  // (axis a, component c, accumulator 0 div / 1 + b omega_b, sign, init)
  struct Pass { int a, c, target; double sign; int init; };
  const Pass passes[9] = {
      {0, 0, 0, 1.0, 1}, {0, 1, 3, 1.0, 1}, {0, 2, 2, -1.0, 1},   // div; omega_z += d_x v; omega_y -= d_x w
      {1, 0, 3, -1.0, 0}, {1, 1, 0, 1.0, 0}, {1, 2, 1, 1.0, 1},   // omega_z -= d_y u; div; omega_x += d_y w
      {2, 0, 2, 1.0, 0}, {2, 1, 1, -1.0, 0}, {2, 2, 0, 1.0, 0}};  // omega_y += d_z u; omega_x -= d_z v; div
  // With 512-point lines along y and z the eps sums ride on the passes that
  // complete each field (omega_z in the second y pass, omega_y, omega_x and
  // div u in the z passes), which add mu field^2 to the block partials instead
  // of storing the field; the first of them initialises the partials' eps fields.
  const bool fuse_eps = g.ny == 512 && g.nz == 512 && CNSF_DERIV_512;
  int first_sum = 1;
  for (const Pass& ps : passes) {
    DerivAxis da{};
    da.n = dims[ps.a];
    da.stride = strides[ps.a];
    da.nlines = (uint32_t)(N / da.n);
    uint32_t lg = 0;
    while ((1u << lg) < da.n) ++lg;
    da.log2n = ((1u << lg) == da.n && da.n >= 2) ? lg : 0;
    // LDS: one (FFT) or two (direct) complex rows per line pair, plus the
    // twiddle table (FFT) or the derivative kernel (direct), <= 64 KiB
    const uint32_t rows = da.log2n ? 1u : 2u;
    const uint32_t extra = da.log2n ? (da.n - 1) * 16u : (da.n + 2) * 8u;
    uint32_t tp = ((uint32_t)CNSF_DERIV_LDS - extra) / (rows * lds_line(da.n) * 16u);
    if (ps.a == 0 && CNSF_DERIV_PAIRS_X > 0 && (uint32_t)CNSF_DERIV_PAIRS_X < tp) tp = CNSF_DERIV_PAIRS_X;
    if (ps.a != 0 && CNSF_DERIV_PAIRS_YZ > 0 && (uint32_t)CNSF_DERIV_PAIRS_YZ < tp) tp = CNSF_DERIV_PAIRS_YZ;
    da.pairs_per_block = tp < 1 ? 1 : (tp > 16 ? 16 : tp);
    da.axis = ps.a;
    da.init = ps.init;
    da.sign = ps.sign;
    da.kscale = 2.0 * M_PI / ((double)da.n * dx);
    const size_t lds = (size_t)rows * da.pairs_per_block * lds_line(da.n) * sizeof(double2) + extra;
    const int k = (int)(&ps - passes);
    if (fuse_eps && (k == 3 || k >= 6)) {
      da.eps = first_sum ? (full ? 2 : 3) : 1;
      da.eps_d = ps.target == 0;
      first_sum = 0;
    }
    if (da.n == 512 && CNSF_DERIV_512 && da.eps)
      hipLaunchKernelGGL(k_deriv512<true>, dim3(DIAG_BLOCKS), dim3(64 * W512), 0, s, fields + ps.c * N,
                         fields + (4 + ps.target) * N, g, da, (const double*)fields, partials);
    else if (da.n == 512 && CNSF_DERIV_512)
      hipLaunchKernelGGL(k_deriv512<false>, dim3(DIAG_BLOCKS), dim3(64 * W512), 0, s, fields + ps.c * N,
                         fields + (4 + ps.target) * N, g, da, (const double*)fields, partials);
    else
      hipLaunchKernelGGL(k_deriv_axis, dim3(DIAG_BLOCKS), dim3(DB), lds, s, fields + ps.c * N,
                         fields + (4 + ps.target) * N, g, da);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (fuse_eps) return hipSuccess;
  hipLaunchKernelGGL(k_eps_sums, dim3(DIAG_BLOCKS), dim3(DB), 0, s, fields, g, partials, full ? 1 : 0);
  return hipGetLastError();
}

uint32_t spectrum_shells(uint32_t n) {
  const double m = (double)(n / 2);
  return (uint32_t)std::floor(std::sqrt(3.0 * m * m) + 0.5) + 1u;
}

hipError_t launch_spectrum(const Geom& g, double* fields, double* partial, double* E, uint32_t nout, hipStream_t s) {
  const uint32_t n = g.nx;
  const uint64_t N = g.ncells;
  const uint32_t nshells = spectrum_shells(n);
  double2* data = (double2*)(fields + 4 * N);
  double* energy = fields + 6 * N;
  const uint32_t strides[3] = {1u, g.nx, g.nxy};
  uint32_t lg = 0;
  while ((1u << lg) < n) ++lg;
  const uint32_t log2n = ((1u << lg) == n && n >= 2) ? lg : 0;
  const uint32_t rows = log2n ? 1u : 2u;
  const uint32_t extra = log2n ? (n - 1) * 16u : 0u;   // twiddle table
  uint32_t tl = (65536u - extra) / (rows * lds_line(n) * 16u);
  tl = tl < 1 ? 1 : (tl > 16 ? 16 : tl);
  const double n3 = (double)N;
  for (int c = 0; c < 3; ++c) {
    for (int a = 0; a < 3; ++a) {
      SpecAxis sa{};
      sa.n = n;
      sa.stride = strides[a];
      sa.nlines = (uint32_t)(N / n);
      const uint32_t cap = a == 0 ? (uint32_t)CNSF_SPEC_LINES_X : (uint32_t)CNSF_SPEC_LINES_YZ;
      sa.lines_per_block = (cap > 0 && cap < tl) ? cap : tl;
      sa.log2n = log2n;
      sa.axis = a;
      sa.mode = a;
      sa.accumulate = c > 0;
      sa.escale = 0.5 / (n3 * n3);
      const size_t lds_a = (size_t)rows * sa.lines_per_block * lds_line(n) * sizeof(double2) + extra;
      if (n == 512 && CNSF_DERIV_512)
        hipLaunchKernelGGL(k_spectrum512, dim3(DIAG_BLOCKS), dim3(64 * W512), 0, s, fields + c * N, data, energy, g,
                           sa);
      else
        hipLaunchKernelGGL(k_spectrum_axis, dim3(DIAG_BLOCKS), dim3(DB), lds_a, s, fields + c * N, data, energy, g,
                           sa);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_shell_partials, dim3(n), dim3(DB), 4 * nshells * sizeof(double), s, energy, n, nshells, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_shell_final, dim3((nout + 255) / 256), dim3(256), 0, s, partial, n, nshells, nout, E);
  return hipGetLastError();
}

hipError_t launch_diag_final(DiagPartial* partials, int nparts, DiagPartial* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DB), 0, s, partials, nparts, out);
  return hipGetLastError();
}

hipError_t launch_diag_final2(DiagPartial* partials, int nparts, DiagPartial* tmp, int ntmp, DiagPartial* out,
                              hipStream_t s) {
  if (!tmp || ntmp < 1 || nparts <= 4 * DB) return launch_diag_final(partials, nparts, out, s);
  const int nb = std::min(ntmp, (nparts + 4 * DB - 1) / (4 * DB));
  const int chunk = (nparts + nb - 1) / nb;
  hipLaunchKernelGGL(k_diag_chunks, dim3(nb), dim3(DB), 0, s, partials, nparts, chunk, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_diag_final(tmp, nb, out, s);
}

}  // namespace cnsf
