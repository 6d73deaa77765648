// Internal definitions of the cnsf library: lattice constants passed to the
// kernels, population storage codecs, the per-cell physics of the
// relaxed-flux compressible Navier-Stokes-Fourier scheme and the in-place
// streaming addresses.
//
// Per cell (Section 2.2): Q_k = sum_i f_{k,i}; primitives from the ideal gas of
// Section 2.1; fluxes Phi_k of Eq. (2); equilibrium
// f^eq_{k,i} = w_i (Q_k + c_i . Phi_k / (c_s^2 lambda)) with c_s^2 = 1/4 and
// w = (1/4, 1/8 x 6) on D3Q7; BGK update f* = f + omega (f^eq - f) + w_i dt S_k.
// The rate omega follows Eqs. (3)-(6) of Section 2.3.
//
// Populations are stored shifted by the equilibrium of a reference gas at
// rest: g = f - f^eq(Q_ref) (divided by a power-of-two scale s_k for the
// 16-bit formats).  The FP32 update works on g throughout: dQ = sum_i g,
// dp = (gamma-1)(dE - rho|u|^2/2), and g* = g + omega((f^eq - f^eq_ref) - g)
// + w_i dt S, so rounding scales with the deviation, not the absolute value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace cnsf {

constexpr int NC = 14;   // components
constexpr int NV = 7;    // D3Q7 velocities: 0, +x, -x, +y, -y, +z, -z
constexpr int NP = 98;   // populations per cell

// Population layout: component k owns one region of `cstride` elements.  The
// region is cut into groups of SLOT_GROUP consecutive cells; a group holds
// the 7 slots one after the other, SLOT_GROUP elements each, cells in linear
// order (x fastest).  A wavefront of 64 consecutive cells therefore reads 64
// consecutive elements of each slot, and a block's tile reads 7 contiguous
// runs per component instead of 98 widely separated streams.
constexpr uint32_t SLOT_GROUP_LOG2 = 10;
constexpr uint32_t SLOT_GROUP = 1u << SLOT_GROUP_LOG2;

// Lattice geometry and boundary data (kernel argument).
struct Geom {
  uint32_t nx, ny, nz, nxy, ncells;
  uint32_t pad_;
  uint64_t cstride;        // elements between the regions of consecutive components
  int32_t bc_x;            // 0 periodic, 1 parity wall, 2 equilibrium ends, 3 no-slip wall
  float dev_left[NC];      // f^eq_{k,+x}(Q_left) - f^eq_{k,+x}(Q_ref): enters at x = 0
  float dev_right[NC];     // f^eq_{k,-x}(Q_right) - f^eq_{k,-x}(Q_ref): enters at x = nx-1
  // no-slip walls, [0] at x = 0 and [1] at x = nx-1: tangential velocity,
  // isothermal flag, and for isothermal walls nu_R(T_w) and K_q(T_w) T_w - (K_q T)_ref
  float wall_uy[2], wall_uz[2], wall_nuR[2], wall_dKT[2];
  int32_t wall_iso[2];
};

// Physical constants of the update, in the precision of the arithmetic.
template <typename R>
struct PhysT {
  R four_over_lam;   // 1 / (c_s^2 lambda) = 4 dt / dx
  R dt;
  R gm1;             // gamma - 1
  R mu0;
  R inv_Tref;
  R visc_param;
  int32_t visc_law;  // 0 const, 1 Sutherland, 2 power
  R inv_tauR, inv_tauq;
  R kq_over_mu0;     // kappa / (mu0 tau_q): K_q = kq_over_mu0 * mu_T
  R three_tauR_4;    // 3 tau_R / 4
  R fmu_coef;        // 4 f_mu dt / dx^2: tau_base = 1/2 + fmu_coef mu_T / rho
  R tb_override;     // > 0: constant tau_base
  R C_sigma, J_min, omega_min;
};
using Phys = PhysT<float>;
using PhysD = PhysT<double>;

// Reference state Q_ref = (rho_ref, 0, 0, 0, E_ref, 0, ...), a gas at rest.
// Its equilibrium is w_i Q_ref,k plus +-fm along the axis of rho u_a (the
// pressure) and +-fq along the axis of q_a (the K_q T term).
struct Codec {
  float rho_w;    // rho_ref
  float E_w;      // E_ref
  float fm;       // w_1 p_ref / (c_s^2 lambda)
  float fq;       // w_1 (K_q T)_ref / (c_s^2 lambda)
  float KT_ref;   // (K_q T)_ref
  float scale[NC];
  float inv_scale[NC];
  int32_t scaled;  // some s_k != 1: the kernels multiply by s_k / 1/s_k
};

// f^eq_{k,i}(Q_ref) (k, i compile-time after unrolling).
template <typename R>
__host__ __device__ inline R feq_ref(const Codec& cd, int k, int i) {
  const R w = i == 0 ? R(0.25) : R(0.125);
  if (k == 0) return w * (R)cd.rho_w;
  if (k == 4) return w * (R)cd.E_w;
  if (i == 0) return R(0);
  const int ax = (i - 1) >> 1;
  const R sg = (i & 1) ? R(1) : R(-1);
  if (k >= 1 && k <= 3 && ax == k - 1) return sg * (R)cd.fm;
  if (k >= 11 && ax == k - 11) return sg * (R)cd.fq;
  return R(0);
}

template <typename R>
__host__ __device__ inline R q_ref(const Codec& cd, int k) {
  return k == 0 ? (R)cd.rho_w : (k == 4 ? (R)cd.E_w : R(0));
}

// ------------------------------------------------------------------ storage
template <int ST>
struct Store;
template <>
struct Store<0> {
  using T = float;
  __device__ static inline float dec(float v) { return v; }
  __device__ static inline float enc(float x) { return x; }
};
template <>
struct Store<1> {  // IEEE binary16, round to nearest even
  using T = uint16_t;
  __device__ static inline float dec(uint16_t v) { return (float)__builtin_bit_cast(_Float16, v); }
  __device__ static inline uint16_t enc(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
};
template <>
struct Store<2> {  // bfloat16, round to nearest even (native conversion on gfx950)
  using T = uint16_t;
  __device__ static inline float dec(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }
  __device__ static inline uint16_t enc(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
};

// ------------------------------------------------------------------ D3Q7
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// component of tau_ab
__host__ __device__ constexpr int tau_idx(int a, int b) {
  return (a == b) ? 5 + a : ((a + b == 1) ? 8 : ((a + b == 2) ? 9 : 10));
}
// (a, b) of stress component K = 5..10
__host__ __device__ constexpr int tau_a(int K) { return (K <= 7) ? K - 5 : (K == 10 ? 1 : 0); }
__host__ __device__ constexpr int tau_b(int K) { return (K <= 7) ? K - 5 : (K == 8 ? 1 : 2); }
// components odd under x -> -x: rho u_x, tau_xy, tau_xz, q_x
__host__ __device__ constexpr bool x_odd(int k) { return k == 1 || k == 8 || k == 9 || k == 11; }

// ------------------------------------------------------------------ physics
template <typename R>
struct Prim {
  R rho, inv_rho, u[3], E, p, T, muT, nuR, Kq;
};

template <typename R>
__host__ __device__ inline R visc_ratio(R th, int law, R param) {
  if (law == 1) return (R(1) + param) * th * sqrt(th) / (th + param);
  if (law == 2) return pow(th, param);
  return R(1);
}
__device__ inline float visc_ratio_f(float th, int law, float param) {
  if (law == 1) return (1.0f + param) * th * __builtin_sqrtf(th) / (th + param);
  if (law == 2) return __builtin_exp2f(param * __builtin_log2f(th));
  return 1.0f;
}

template <typename R>
__host__ __device__ inline R mu_of_T(R T, const PhysT<R>& ph) {
#ifdef __HIP_DEVICE_COMPILE__
  if constexpr (sizeof(R) == 4) return ph.mu0 * visc_ratio_f(T * ph.inv_Tref, ph.visc_law, ph.visc_param);
#endif
  return ph.mu0 * visc_ratio<R>(T * ph.inv_Tref, ph.visc_law, ph.visc_param);
}

template <typename R>
__host__ __device__ inline Prim<R> primitives(const R Q[NC], const PhysT<R>& ph) {
  Prim<R> P;
  P.rho = Q[0];
  P.inv_rho = R(1) / P.rho;
  P.u[0] = Q[1] * P.inv_rho;
  P.u[1] = Q[2] * P.inv_rho;
  P.u[2] = Q[3] * P.inv_rho;
  P.E = Q[4];
  P.p = ph.gm1 * (P.E - R(0.5) * (Q[1] * P.u[0] + Q[2] * P.u[1] + Q[3] * P.u[2]));
  P.T = P.p * P.inv_rho;
  P.muT = mu_of_T<R>(P.T, ph);
  P.nuR = P.muT * ph.inv_tauR;
  P.Kq = ph.kq_over_mu0 * P.muT;
  return P;
}

// Flux of component K along the three axes (Eq. (2) sign convention).  The
// momentum groups take `p_term` for the pressure and the heat-flux groups
// `KT_term` for K_q T; passing p - p_ref and K_q T - (K_q T)_ref gives the
// flux less the reference state's flux.
template <int K, typename R>
__host__ __device__ inline void flux(const R Q[NC], const R u[3], R E_plus_p, R p_term, R nuR, R KT_term, R phi[3]) {
  if constexpr (K == 0) {
    phi[0] = Q[1];
    phi[1] = Q[2];
    phi[2] = Q[3];
  } else if constexpr (K >= 1 && K <= 3) {
    constexpr int a = K - 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) phi[c] = Q[K] * u[c] - Q[tau_idx(a, c)];
    phi[a] += p_term;
  } else if constexpr (K == 4) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      phi[c] = E_plus_p * u[c] - (Q[tau_idx(c, 0)] * u[0] + Q[tau_idx(c, 1)] * u[1] + Q[tau_idx(c, 2)] * u[2]) + Q[11 + c];
  } else if constexpr (K >= 5 && K <= 10) {
    constexpr int a = tau_a(K), b = tau_b(K);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R lam = R(0);
      if (b == c) lam += u[a];
      if (a == c) lam += u[b];
      if (a == b) lam -= R(2) / R(3) * u[c];
      phi[c] = Q[K] * u[c] - nuR * lam;
    }
  } else {
    constexpr int a = K - 11;
#pragma unroll
    for (int c = 0; c < 3; ++c) phi[c] = Q[K] * u[c];
    phi[a] += KT_term;
  }
}

// Absolute equilibrium of every component (FP64 initialisation, host tables).
template <typename R>
__host__ __device__ inline void equilibrium_all(const R Q[NC], const Prim<R>& P, R four_over_lam, R feq[NC][NV]) {
  R phi[NC][3];
  const R Ep = P.E + P.p, KT = P.Kq * P.T;
  flux<0, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[0]);
  flux<1, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[1]);
  flux<2, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[2]);
  flux<3, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[3]);
  flux<4, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[4]);
  flux<5, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[5]);
  flux<6, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[6]);
  flux<7, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[7]);
  flux<8, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[8]);
  flux<9, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[9]);
  flux<10, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[10]);
  flux<11, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[11]);
  flux<12, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[12]);
  flux<13, R>(Q, P.u, Ep, P.p, P.nuR, KT, phi[13]);
  for (int k = 0; k < NC; ++k) {
    feq[k][0] = R(0.25) * Q[k];
    for (int a = 0; a < 3; ++a) {
      const R d = four_over_lam * phi[k][a];
      feq[k][1 + 2 * a] = R(0.125) * (Q[k] + d);
      feq[k][2 + 2 * a] = R(0.125) * (Q[k] - d);
    }
  }
}

// Relaxation rate of the cell, Eqs. (3)-(6).  The dilatation is read from the
// normal-stress groups: for axis a, f_{+a} + f_{-a} - f_0 of tau_aa equals its
// non-equilibrium combination (the equilibrium part cancels since
// 2 w_1 = w_0; the reference shift of these groups is zero), which is
// -tau_base dt d_a Phi_{tau_aa,a} to first order, and sum_a Phi_{tau_aa,a}
// carries -(4/3)(mu_T/tau_R) div u.  `g` may hold f or f - f^eq(Q_ref).
// Returns omega_h; *chi_out (if given) receives chi.
template <typename R>
__host__ __device__ inline R relaxation_rate(const R g[NC][NV], R muT, R inv_rho, const PhysT<R>& ph,
                                             R* chi_out = nullptr) {
  const R tb = ph.tb_override > R(0) ? ph.tb_override : R(0.5) + ph.fmu_coef * muT * inv_rho;
  const R omega_b = R(1) / tb;
  R chi = R(0);
  if (ph.C_sigma > R(0)) {
    const R nsum = (g[5][1] + g[5][2] - g[5][0]) + (g[6][3] + g[6][4] - g[6][0]) + (g[7][5] + g[7][6] - g[7][0]);
    // theta = dt div u = -(3 tau_R / (4 mu_T)) sum_a D_a,  D_a = -(...)/tau_base
    const R theta = ph.three_tauR_4 * nsum / (tb * muT);
    const R s = (theta < R(0) ? -theta : R(0)) * R(2);   // / c_s, c_s = 1/2
    if (s > ph.J_min) chi = (ph.C_sigma * s < R(1)) ? ph.C_sigma * s : R(1);
  }
  if (chi_out) *chi_out = chi;
  const R drop = omega_b > ph.omega_min ? omega_b - ph.omega_min : R(0);
  return omega_b - chi * drop;
}

// Primitives of the shifted state (FP32 update).
struct DevPrim {
  float rho, inv_rho, u[3], E_plus_p, dp, T, muT, nuR, dKT;
};

// Fill dQ, Q and P from shifted populations; returns the cell's relaxation rate.
__device__ inline float cell_state(const float g[NC][NV], const Codec& cd, const Phys& ph, float dQ[NC], float Q[NC],
                                   DevPrim& P, float* chi_out = nullptr) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    dQ[k] = ((g[k][0] + g[k][1]) + (g[k][2] + g[k][3])) + ((g[k][4] + g[k][5]) + g[k][6]);
    Q[k] = dQ[k];
  }
  Q[0] += cd.rho_w;
  Q[4] += cd.E_w;
  P.rho = Q[0];
  P.inv_rho = 1.0f / P.rho;
  P.u[0] = Q[1] * P.inv_rho;
  P.u[1] = Q[2] * P.inv_rho;
  P.u[2] = Q[3] * P.inv_rho;
  const float ke = 0.5f * (Q[1] * P.u[0] + Q[2] * P.u[1] + Q[3] * P.u[2]);
  P.dp = ph.gm1 * (dQ[4] - ke);                 // p - p_ref, p_ref = (gamma-1) E_ref
  const float p = ph.gm1 * cd.E_w + P.dp;
  P.E_plus_p = Q[4] + p;
  P.T = p * P.inv_rho;
  P.muT = mu_of_T<float>(P.T, ph);
  P.nuR = P.muT * ph.inv_tauR;
  P.dKT = ph.kq_over_mu0 * P.muT * P.T - cd.KT_ref;
  return relaxation_rate<float>(g, P.muT, P.inv_rho, ph, chi_out);
}

// BGK collision of component K on the shifted populations, in place:
// g <- g + omega ((f^eq - f^eq_ref) - g) + w_i dt S_K.
template <int K>
__device__ inline void collide_dev(float g[NV], const float dQ[NC], const float Q[NC], const DevPrim& P, const Phys& ph,
                                   float omega) {
  float phi[3];
  flux<K, float>(Q, P.u, P.E_plus_p, P.dp, P.nuR, P.dKT, phi);
  float S = 0.0f;
  if constexpr (K >= 5) S = -dQ[K] * (K <= 10 ? ph.inv_tauR : ph.inv_tauq);
  const float s0 = 0.25f * ph.dt * S, s1 = 0.125f * ph.dt * S;
  g[0] += omega * (0.25f * dQ[K] - g[0]) + s0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float e = ph.four_over_lam * phi[a];
    g[1 + 2 * a] += omega * (0.125f * (dQ[K] + e) - g[1 + 2 * a]) + s1;
    g[2 + 2 * a] += omega * (0.125f * (dQ[K] - e) - g[2 + 2 * a]) + s1;
  }
}

// Pre-collision values of a cell that a no-slip wall next to it needs.
struct WallCell {
  float rho, nuR, txy, txz, qx;
};

// The whole cell update on shifted populations (FP32).  `wc`, if given,
// receives the values a no-slip wall takes from the cell.
__device__ inline void update_cell(float g[NC][NV], const Codec& cd, const Phys& ph, float* chi_out = nullptr,
                                   WallCell* wc = nullptr) {
  float dQ[NC], Q[NC];
  DevPrim P;
  const float omega = cell_state(g, cd, ph, dQ, Q, P, chi_out);
  if (wc) {
    wc->rho = P.rho;
    wc->nuR = P.nuR;
    wc->txy = Q[8];
    wc->txz = Q[9];
    wc->qx = Q[11];
  }
  collide_dev<0>(g[0], dQ, Q, P, ph, omega);
  collide_dev<1>(g[1], dQ, Q, P, ph, omega);
  collide_dev<2>(g[2], dQ, Q, P, ph, omega);
  collide_dev<3>(g[3], dQ, Q, P, ph, omega);
  collide_dev<4>(g[4], dQ, Q, P, ph, omega);
  collide_dev<5>(g[5], dQ, Q, P, ph, omega);
  collide_dev<6>(g[6], dQ, Q, P, ph, omega);
  collide_dev<7>(g[7], dQ, Q, P, ph, omega);
  collide_dev<8>(g[8], dQ, Q, P, ph, omega);
  collide_dev<9>(g[9], dQ, Q, P, ph, omega);
  collide_dev<10>(g[10], dQ, Q, P, ph, omega);
  collide_dev<11>(g[11], dQ, Q, P, ph, omega);
  collide_dev<12>(g[12], dQ, Q, P, ph, omega);
  collide_dev<13>(g[13], dQ, Q, P, ph, omega);
}

// ------------------------------------------------------------------ addressing
// Linear neighbours of cell c = (x, y, z) with periodic wrap in all axes.
struct Nbr {
  uint32_t c, xm, xp, ym, yp, zm, zp;
  uint32_t x;
};

__device__ inline Nbr neighbours(uint32_t c, const Geom& g) {
  Nbr n;
  n.c = c;
  const uint32_t x = c % g.nx;
  const uint32_t t = c / g.nx;
  const uint32_t y = t % g.ny;
  const uint32_t z = t / g.ny;
  n.x = x;
  n.xm = (x == 0) ? c + (g.nx - 1) : c - 1;
  n.xp = (x == g.nx - 1) ? c - (g.nx - 1) : c + 1;
  n.ym = (y == 0) ? c + (g.nxy - g.nx) : c - g.nx;
  n.yp = (y == g.ny - 1) ? c - (g.nxy - g.nx) : c + g.nx;
  n.zm = (z == 0) ? c + (g.ncells - g.nxy) : c - g.nxy;
  n.zp = (z == g.nz - 1) ? c - (g.ncells - g.nxy) : c + g.nxy;
  return n;
}

// In-place (AA) streaming.  Even passes read slot i of the cell and write the
// post-collision value to slot opp(i) of the same cell.  Odd passes read
// f_i(x) from slot opp(i) of x - c_i and write f*_i(x) to slot i of x + c_i.
__device__ inline uint32_t odd_src(const Nbr& n, int i) {  // x - c_i
  switch (i) {
    case 1: return n.xm;
    case 2: return n.xp;
    case 3: return n.ym;
    case 4: return n.yp;
    case 5: return n.zm;
    case 6: return n.zp;
    default: return n.c;
  }
}

// Element index, inside one component's region, of slot `slot` of cell `idx`.
__host__ __device__ inline uint32_t slot_index(int slot, uint32_t idx) {
  return (idx >> SLOT_GROUP_LOG2) * (uint32_t)(NV * SLOT_GROUP) + (uint32_t)slot * SLOT_GROUP + (idx & (SLOT_GROUP - 1u));
}

// Byte offset of the same element.  A component's region spans less than
// 4 GiB (checked on the host).
template <int ST>
__device__ inline uint32_t slot_offset(const Geom&, int slot, uint32_t idx) {
  return slot_index(slot, idx) * (uint32_t)sizeof(typename Store<ST>::T);
}

// Raw buffer access to one component's region: a 128-bit resource (base,
// byte size) in scalar registers plus one 32-bit offset per direction.  The
// hardware drops accesses at or past the size (reads return 0).
constexpr int BUF_WORD3 = 0x00020000;   // gfx9-family resource word 3

template <int ST>
__device__ inline __amdgpu_buffer_rsrc_t component_rsrc(const typename Store<ST>::T* pop, const Geom& g, int k) {
  const uint32_t bytes = (uint32_t)(g.cstride * sizeof(typename Store<ST>::T));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(pop + (uint64_t)k * g.cstride), (short)0, (int)bytes, BUF_WORD3);
}

template <int ST>
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (ST == 0) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  } else {
    return Store<ST>::dec((uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
  }
}

template <int ST>
__device__ inline void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  if constexpr (ST == 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, (int)off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16((short)Store<ST>::enc(v), r, (int)off, 0, 0);
  }
}

// True where link i of the current time level crossed an x-end in the last
// odd pass: the reads of i = +x at x = 0 and of i = -x at x = nx - 1.
template <int BC>
__device__ inline bool crossed_end(const Geom& g, const Nbr& n, int parity, int i) {
  return BC != 0 && parity && ((i == 1 && n.x == 0) || (i == 2 && n.x == g.nx - 1));
}

// The 7 byte offsets (within one component's region) from which the current
// time level's f_i is read.  Even passes: slot i of the cell.  Odd passes:
// slot opp(i) of x - c_i, or, for a link that crossed an x-end, slot i of the
// cell itself (where the previous even pass left the post-collision value of
// opp(i)).  The update writes f*_i back to off[opp(i)]: each thread writes
// exactly the 98 addresses it read, so a pass is race free in place.
template <int ST, int BC>
__device__ inline void stream_offsets(const Geom& g, const Nbr& n, int parity, uint32_t off[NV]) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    int slot = parity ? opp(i) : i;
    uint32_t idx = parity ? odd_src(n, i) : n.c;
    if (crossed_end<BC>(g, n, parity, i)) {
      slot = i;
      idx = n.c;
    }
    off[i] = slot_offset<ST>(g, slot, idx);
  }
}

// Gather the 98 shifted populations g = f - f^eq(Q_ref) of the current time
// level.  BC: 0 periodic, 1 parity wall, 2 equilibrium ends, 3 no-slip wall.
// A link that crossed a parity wall returns reversed with the mirror sign of
// its component; the reference shift is mirror-symmetric in x, so the shifted
// value simply changes sign for the x-odd components.  At an equilibrium end
// the link is the end state's equilibrium.  At a no-slip wall the emitting
// cell already stored the returned link.
template <int ST, int BC, bool SC, typename R>
__device__ inline void gather(const typename Store<ST>::T* __restrict__ pop, const Geom& g, const Codec& cd,
                              const Nbr& n, int parity, const uint32_t off[NV], R gv[NC][NV]) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const __amdgpu_buffer_rsrc_t rs = component_rsrc<ST>(pop, g, k);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R v = (R)buf_load<ST>(rs, off[i]);
      if (ST != 0 && SC) v *= (R)cd.scale[k];
      if (crossed_end<BC>(g, n, parity, i)) {
        if (BC == 1 && x_odd(k)) v = -v;
        if (BC == 2) v = (R)(i == 1 ? g.dev_left[k] : g.dev_right[k]);
      }
      gv[k][i] = v;
    }
  }
}

// No-slip wall: side (0 at x = 0, 1 at x = nx-1) through which the cell emits
// link i, or -1.  The emitting cell turns the link round in both passes; the
// next pass reads it back unchanged.
template <int BC>
__device__ inline int noslip_side(const Geom& g, const Nbr& n, int i) {
  if (BC != 3) return -1;
  if (i == 2 && n.x == 0) return 0;
  if (i == 1 && n.x == g.nx - 1) return 1;
  return -1;
}

// The link of component k returning from no-slip wall s, in shifted form, from
// the outgoing g*.  The wall fixes the momentum (rho u_w) and, when adiabatic,
// q_x = 0: anti-bounce-back, f_in = -f*_out + 2 w_1 Q_w.  Every other component
// returns with the normal flux of Eq. (2) at the wall state (the cell's rho,
// tau, q; the wall's velocity; T_w when isothermal): f_in = f*_out +
// 2 w_1 c_in Phi_w / (c_s^2 lambda).  The reference shift cancels except in
// q_x's flux, hence K_q T_w - (K_q T)_ref.
__device__ inline float noslip_link(int k, float v, int s, const Geom& g, const Phys& ph, const WallCell& w) {
  const float F = (s == 0 ? 0.25f : -0.25f) * ph.four_over_lam;   // 2 w_1 c_in / (c_s^2 lambda)
  const bool iso = g.wall_iso[s] != 0;
  const float uy = g.wall_uy[s], uz = g.wall_uz[s];
  const float nuR = iso ? g.wall_nuR[s] : w.nuR;
  switch (k) {
    case 1: return -v;
    case 2: return -v + 0.25f * w.rho * uy;
    case 3: return -v + 0.25f * w.rho * uz;
    case 4: return v + F * ((iso ? w.qx : 0.0f) - (w.txy * uy + w.txz * uz));
    case 8: return v - F * nuR * uy;
    case 9: return v - F * nuR * uz;
    case 11: return iso ? v + F * g.wall_dKT[s] : -v;
    default: return v;
  }
}

// Write g*_i to off[opp(i)] (see stream_offsets).  A link leaving through an
// x-end is stored back into the cell as the opposite direction: mirrored at a
// parity wall, replaced by the end state's equilibrium at an equilibrium end,
// turned round by the no-slip rule (`ph`, `w` used only there).
template <int ST, int BC, bool SC>
__device__ inline void scatter(typename Store<ST>::T* __restrict__ pop, const Geom& g, const Codec& cd,
                               const Phys& ph, const WallCell& w, const Nbr& n, int parity, const uint32_t off[NV],
                               const float gv[NC][NV]) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const __amdgpu_buffer_rsrc_t rs = component_rsrc<ST>(pop, g, k);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      float v = gv[k][i];
      if (BC == 1 || BC == 2) {
        if (crossed_end<BC>(g, n, parity, opp(i))) {
          if (BC == 1 && x_odd(k)) v = -v;
          if (BC == 2) v = (i == 2) ? g.dev_left[k] : g.dev_right[k];
        }
      }
      if (BC == 3) {
        const int s = noslip_side<BC>(g, n, i);
        if (s >= 0) v = noslip_link(k, v, s, g, ph, w);
      }
      if (ST != 0 && SC) v *= cd.inv_scale[k];
      buf_store<ST>(rs, off[opp(i)], v);
    }
  }
}

}  // namespace cnsf
