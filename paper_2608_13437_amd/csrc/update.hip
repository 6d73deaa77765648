// Fused stream-and-collide update, state initialisation and moment readout.
//
// One thread owns one cell.  Populations live in 14 component regions, each
// cut into groups of 1024 consecutive cells that hold the 7 slots back to
// back (x fastest inside a slot), so a wavefront of 64 consecutive cells
// reads 64 consecutive elements of every slot.  The in-place AA pattern
// alternates an even pass (read and write the cell's own slots) and an odd
// pass (read from and write to the six face neighbours), so one array holds
// the whole lattice.
#include "cnsf_impl.h"
#include "diag_common.h"
#include "launch.h"

namespace cnsf {

// Tile index remap: hardware deals blocks round-robin over the 8 XCDs; this
// gives XCD j one contiguous span of tiles so that the cache lines shared by
// neighbouring tiles (the +-x halo of the odd pass) stay in one L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / 8u, rem = nb % 8u;
  const uint32_t j = b % 8u, q = b / 8u;
  return j * per + (j < rem ? j : rem) + q;
}

// One block owns a tile of `tile` consecutive cells and walks it blockDim
// cells at a time (so each wave streams through consecutive segments of
// every slot).  With one block per tile the remap hands XCD j a contiguous
// span of tiles; with a persistent grid (fewer blocks than tiles, a multiple
// of 8) the blocks of XCD j stride over the j-th eighth of the tiles, so
// neighbouring tiles, which share the +-x halo lines of the odd pass, are in
// flight in the same L2.  Without the remap the blocks stride over all tiles.
//
// DIAG instances also reduce the Eq. (7) sums of the time level they read
// (one partial per block, as the diagnostics readout forms them) and, when
// `fields` is given, write u, v, w, mu for the spectral derivatives.
template <int ST, int BC, bool SC, int PAR, bool DIAG>
__global__ void __launch_bounds__(256) k_update(typename Store<ST>::T* __restrict__ pop, const Geom g, const Phys ph,
                                                const Codec cd, uint32_t tile, uint32_t ntiles, int remap,
                                                const PhysD phd, DiagPartial* __restrict__ partials,
                                                double* __restrict__ fields) {
  constexpr int parity = PAR;
  DiagPartial acc;
  if constexpr (DIAG) part_zero(acc);
  uint32_t t_begin = blockIdx.x, t_step = gridDim.x, t_end = ntiles;
  if (remap && gridDim.x >= ntiles) {
    t_begin = xcd_block(blockIdx.x, ntiles);
    t_end = t_begin + 1;
  } else if (remap && (gridDim.x & 7u) == 0) {
    const uint32_t per = (ntiles + 7u) / 8u, x = blockIdx.x & 7u;
    t_begin = x * per + (blockIdx.x >> 3);
    t_step = gridDim.x >> 3;
    t_end = min(ntiles, (x + 1u) * per);
  }
  for (uint32_t t = t_begin; t < t_end; t += t_step) {
    const uint32_t first = t * tile;
    for (uint32_t j = threadIdx.x; j < tile; j += blockDim.x) {
      const uint32_t c = first + j;
      if (c >= g.ncells) break;
      const Nbr n = neighbours(c, g);
      uint32_t off[NV];
      stream_offsets<ST, BC>(g, n, parity, off);
      float gv[NC][NV];
      gather<ST, BC, SC, float>(pop, g, cd, n, parity, off, gv);
      WallCell wc{};
      if constexpr (DIAG) {
        cell_sums(gv, cd, phd, c, g.ncells, fields, acc);
        float chi = 0.0f;
        update_cell(gv, cd, ph, &chi, BC == 3 ? &wc : nullptr);
        acc.sensor += chi > 0.0f ? 1.0 : 0.0;
      } else {
        update_cell(gv, cd, ph, nullptr, BC == 3 ? &wc : nullptr);
      }
      scatter<ST, BC, SC>(pop, g, cd, ph, wc, n, parity, off, gv);
    }
  }
  if constexpr (DIAG) {
    const DiagPartial tot = block_reduce(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

// f = f^eq(Q) for cells of z-planes [z0, z0 + nzs); FP64 arithmetic.  With
// PRIM the input holds rho, u (3), p, tau (6), q (3) per cell, turned into the
// conserved state (ideal gas, Section 2.1) first.
template <int ST, bool PRIM>
__global__ void k_init(typename Store<ST>::T* __restrict__ pop, const double* __restrict__ Q, const Geom g,
                       const PhysD ph, const Codec cd, uint32_t cell0, uint32_t nslab, int* __restrict__ bad) {
  using S = Store<ST>;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslab) return;
  const uint32_t c = cell0 + j;
  double q[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) q[k] = Q[(uint64_t)k * nslab + j];
  if (PRIM) {
    const double rho = q[0], ux = q[1], uy = q[2], uz = q[3], p = q[4];
    q[1] = rho * ux;
    q[2] = rho * uy;
    q[3] = rho * uz;
    q[4] = p / ph.gm1 + 0.5 * rho * (ux * ux + uy * uy + uz * uz);
  }
  Prim<double> P = primitives<double>(q, ph);
  bool ok = P.rho > 0.0 && P.p > 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) ok = ok && isfinite(q[k]);
  if (!ok) atomicOr(bad, 1);
  double feq[NC][NV];
  equilibrium_all<double>(q, P, ph.four_over_lam, feq);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    typename S::T* base = pop + slot_index(i, c);
#pragma unroll
    for (int k = 0; k < NC; ++k)
      base[k * g.cstride] = S::enc((float)((feq[k][i] - feq_ref<double>(cd, k, i)) * (double)cd.inv_scale[k]));
  }
}

// rho, u (3), p, T of the current time level (FP64, from the FP64 moments).
template <int ST, int BC>
__global__ void k_primitives(const typename Store<ST>::T* __restrict__ pop, double* __restrict__ out, const Geom g,
                             const Codec cd, const PhysD ph, int parity, uint32_t cell0, uint32_t nslab) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslab) return;
  const Nbr n = neighbours(cell0 + j, g);
  uint32_t off[NV];
  stream_offsets<ST, BC>(g, n, parity, off);
  float gf[NC][NV];
  gather<ST, BC, true, float>(pop, g, cd, n, parity, off, gf);
  double Q[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) s += (double)gf[k][i];
    Q[k] = q_ref<double>(cd, k) + s;
  }
  const Prim<double> P = primitives<double>(Q, ph);
  const double v[6] = {P.rho, P.u[0], P.u[1], P.u[2], P.p, P.T};
#pragma unroll
  for (int k = 0; k < 6; ++k) out[(uint64_t)k * nslab + j] = v[k];
}

// Q_k = sum_i f_{k,i} of the current time level (FP64 accumulation).
template <int ST, int BC>
__global__ void k_moments(const typename Store<ST>::T* __restrict__ pop, double* __restrict__ out, const Geom g,
                          const Codec cd, int parity, uint32_t cell0, uint32_t nslab) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nslab) return;
  const Nbr n = neighbours(cell0 + j, g);
  uint32_t off[NV];
  stream_offsets<ST, BC>(g, n, parity, off);
  double gv[NC][NV];
  gather<ST, BC, true, double>(pop, g, cd, n, parity, off, gv);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) s += gv[k][i];
    out[(uint64_t)k * nslab + j] = q_ref<double>(cd, k) + s;
  }
}

// Plain copy, 4 x 16 bytes in flight per thread per iteration, non-temporal
// loads and stores (the copy's data is touched once).  Of the variants measured
// on a 26 GB copy inside a fast 52.6 GB allocation on MI355X (1, 4 or 8 vectors
// per thread, temporal or not, grid-strided or block-contiguous, 8 to 64 blocks
// per compute unit) this one, at 64 blocks per unit, moves the most: 6.33 TB/s
// against 5.92 TB/s for temporal accesses.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const u32x4 a = __builtin_nontemporal_load(&src[i]), b = __builtin_nontemporal_load(&src[i + stride]);
    const u32x4 c = __builtin_nontemporal_load(&src[i + 2 * stride]), d = __builtin_nontemporal_load(&src[i + 3 * stride]);
    __builtin_nontemporal_store(a, &dst[i]);
    __builtin_nontemporal_store(b, &dst[i + stride]);
    __builtin_nontemporal_store(c, &dst[i + 2 * stride]);
    __builtin_nontemporal_store(d, &dst[i + 3 * stride]);
  }
  for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

// ------------------------------------------------------------------ launchers
uint32_t update_blocks(const Geom& g, const Launch& lc) {
  const uint32_t ntiles = (g.ncells + lc.tile - 1) / lc.tile;
  return (lc.grid > 0 && (uint32_t)lc.grid < ntiles) ? (uint32_t)lc.grid : ntiles;
}

template <int ST, int BC, bool SC, bool DIAG>
static hipError_t launch_update_t(void* pop, const Geom& g, const Phys& ph, const Codec& cd, int parity,
                                  const Launch& lc, const PhysD& phd, DiagPartial* partials, double* fields,
                                  hipStream_t s) {
  const uint32_t ntiles = (g.ncells + lc.tile - 1) / lc.tile;
  const uint32_t nb = update_blocks(g, lc);
  using T = typename Store<ST>::T;
  if (parity)
    hipLaunchKernelGGL((k_update<ST, BC, SC, 1, DIAG>), dim3(nb), dim3(lc.block), 0, s, (T*)pop, g, ph, cd,
                       (uint32_t)lc.tile, ntiles, lc.remap, phd, partials, fields);
  else
    hipLaunchKernelGGL((k_update<ST, BC, SC, 0, DIAG>), dim3(nb), dim3(lc.block), 0, s, (T*)pop, g, ph, cd,
                       (uint32_t)lc.tile, ntiles, lc.remap, phd, partials, fields);
  return hipGetLastError();
}

hipError_t launch_update(int storage, void* pop, const Geom& g, const Phys& ph, const Codec& cd, int parity,
                         const Launch& lc, hipStream_t s) {
  const bool sc = cd.scaled != 0;
  const PhysD none{};
#define CNSF_CASE(ST, BC, SC)                              \
  if (storage == ST && g.bc_x == BC && sc == SC)           \
    return launch_update_t<ST, BC, SC, false>(pop, g, ph, cd, parity, lc, none, nullptr, nullptr, s);
  CNSF_CASE(0, 0, false) CNSF_CASE(0, 1, false) CNSF_CASE(0, 2, false) CNSF_CASE(0, 3, false)
  CNSF_CASE(1, 0, false) CNSF_CASE(1, 1, false) CNSF_CASE(1, 2, false) CNSF_CASE(1, 3, false)
  CNSF_CASE(2, 0, false) CNSF_CASE(2, 1, false) CNSF_CASE(2, 2, false) CNSF_CASE(2, 3, false)
  CNSF_CASE(1, 0, true) CNSF_CASE(1, 1, true) CNSF_CASE(1, 2, true) CNSF_CASE(1, 3, true)
  CNSF_CASE(2, 0, true) CNSF_CASE(2, 1, true) CNSF_CASE(2, 2, true) CNSF_CASE(2, 3, true)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_update_diag(int storage, void* pop, const Geom& g, const Phys& ph, const Codec& cd, int parity,
                              const Launch& lc, const PhysD& phd, DiagPartial* partials, double* fields,
                              hipStream_t s) {
  const bool sc = cd.scaled != 0;
#define CNSF_CASE(ST, BC, SC)                    \
  if (storage == ST && g.bc_x == BC && sc == SC) \
    return launch_update_t<ST, BC, SC, true>(pop, g, ph, cd, parity, lc, phd, partials, fields, s);
  CNSF_CASE(0, 0, false) CNSF_CASE(0, 1, false) CNSF_CASE(0, 2, false) CNSF_CASE(0, 3, false)
  CNSF_CASE(1, 0, false) CNSF_CASE(1, 1, false) CNSF_CASE(1, 2, false) CNSF_CASE(1, 3, false)
  CNSF_CASE(2, 0, false) CNSF_CASE(2, 1, false) CNSF_CASE(2, 2, false) CNSF_CASE(2, 3, false)
  CNSF_CASE(1, 0, true) CNSF_CASE(1, 1, true) CNSF_CASE(1, 2, true) CNSF_CASE(1, 3, true)
  CNSF_CASE(2, 0, true) CNSF_CASE(2, 1, true) CNSF_CASE(2, 2, true) CNSF_CASE(2, 3, true)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

template <int ST, bool PRIM>
static void init_t(void* pop, const double* Q, const Geom& g, const PhysD& ph, const Codec& cd, uint32_t cell0,
                   uint32_t nslab, int* bad, uint32_t nb, hipStream_t s) {
  hipLaunchKernelGGL((k_init<ST, PRIM>), dim3(nb), dim3(256), 0, s, (typename Store<ST>::T*)pop, Q, g, ph, cd, cell0,
                     nslab, bad);
}

hipError_t launch_init(int storage, void* pop, const double* Q, const Geom& g, const PhysD& ph, const Codec& cd,
                       uint32_t cell0, uint32_t nslab, int* bad, bool primitive, hipStream_t s) {
  const uint32_t nb = (nslab + 255) / 256;
  if (nb == 0) return hipSuccess;
  if (storage == 0) (primitive ? init_t<0, true> : init_t<0, false>)(pop, Q, g, ph, cd, cell0, nslab, bad, nb, s);
  else if (storage == 1) (primitive ? init_t<1, true> : init_t<1, false>)(pop, Q, g, ph, cd, cell0, nslab, bad, nb, s);
  else (primitive ? init_t<2, true> : init_t<2, false>)(pop, Q, g, ph, cd, cell0, nslab, bad, nb, s);
  return hipGetLastError();
}

template <int ST, int BC>
static hipError_t launch_primitives_t(const void* pop, double* out, const Geom& g, const Codec& cd, const PhysD& ph,
                                      int parity, uint32_t cell0, uint32_t nslab, hipStream_t s) {
  const uint32_t nb = (nslab + 255) / 256;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL((k_primitives<ST, BC>), dim3(nb), dim3(256), 0, s, (const typename Store<ST>::T*)pop, out, g, cd,
                     ph, parity, cell0, nslab);
  return hipGetLastError();
}

hipError_t launch_primitives(int storage, const void* pop, double* out, const Geom& g, const Codec& cd, const PhysD& ph,
                             int parity, uint32_t cell0, uint32_t nslab, hipStream_t s) {
#define CNSF_CASE(ST, BC) \
  if (storage == ST && g.bc_x == BC) return launch_primitives_t<ST, BC>(pop, out, g, cd, ph, parity, cell0, nslab, s);
  CNSF_CASE(0, 0) CNSF_CASE(0, 1) CNSF_CASE(0, 2) CNSF_CASE(0, 3)
  CNSF_CASE(1, 0) CNSF_CASE(1, 1) CNSF_CASE(1, 2) CNSF_CASE(1, 3)
  CNSF_CASE(2, 0) CNSF_CASE(2, 1) CNSF_CASE(2, 2) CNSF_CASE(2, 3)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

template <int ST, int BC>
static hipError_t launch_moments_t(const void* pop, double* out, const Geom& g, const Codec& cd, int parity,
                                   uint32_t cell0, uint32_t nslab, hipStream_t s) {
  const int block = 256;
  const uint32_t nb = (nslab + block - 1) / block;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL((k_moments<ST, BC>), dim3(nb), dim3(block), 0, s, (const typename Store<ST>::T*)pop, out, g, cd,
                     parity, cell0, nslab);
  return hipGetLastError();
}

hipError_t launch_moments(int storage, const void* pop, double* out, const Geom& g, const Codec& cd, int parity,
                          uint32_t cell0, uint32_t nslab, hipStream_t s) {
#define CNSF_CASE(ST, BC) \
  if (storage == ST && g.bc_x == BC) return launch_moments_t<ST, BC>(pop, out, g, cd, parity, cell0, nslab, s);
  CNSF_CASE(0, 0) CNSF_CASE(0, 1) CNSF_CASE(0, 2) CNSF_CASE(0, 3)
  CNSF_CASE(1, 0) CNSF_CASE(1, 1) CNSF_CASE(1, 2) CNSF_CASE(1, 3)
  CNSF_CASE(2, 0) CNSF_CASE(2, 1) CNSF_CASE(2, 2) CNSF_CASE(2, 3)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const uint64_t want = (n16 + 255) / 256;
  const uint32_t nb = (uint32_t)(want < (uint64_t)ncu * 64 ? (want ? want : 1) : (uint64_t)ncu * 64);
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n16);
  return hipGetLastError();
}

}  // namespace cnsf
