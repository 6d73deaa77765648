// Host-side launchers of the cnsf kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "cnsf_impl.h"

namespace cnsf {

// Launch shape of the update: threads per block (<= 256), cells per tile (a
// multiple of block), blocks in a persistent grid (0: one block per tile) and
// the XCD-contiguous tile remap.
struct Launch {
  int block = 256;
  int tile = 1024;
  int grid = 0;
  int remap = 1;
};
// Shape measured best on MI355X for each storage type (512^3 Taylor-Green).
Launch default_launch(int storage);

hipError_t launch_update(int storage, void* pop, const Geom& g, const Phys& ph, const Codec& cd, int parity,
                         const Launch& lc, hipStream_t s);
hipError_t launch_init(int storage, void* pop, const double* Q, const Geom& g, const PhysD& ph, const Codec& cd,
                       uint32_t cell0, uint32_t nslab, int* bad, bool primitive, hipStream_t s);
hipError_t launch_primitives(int storage, const void* pop, double* out, const Geom& g, const Codec& cd, const PhysD& ph,
                             int parity, uint32_t cell0, uint32_t nslab, hipStream_t s);
hipError_t launch_moments(int storage, const void* pop, double* out, const Geom& g, const Codec& cd, int parity,
                          uint32_t cell0, uint32_t nslab, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Diagnostics: FP64 sums and the spectral dissipation averages.
struct DiagPartial {
  double mass, mx, my, mz, energy, ek2;  // ek2 = sum rho |u|^2
  double min_rho, min_p;
  double sensor, nonfinite;
  double eps_s, eps_d;                   // sums of mu |curl u|^2 and mu (div u)^2
};
constexpr int DIAG_BLOCKS = 2048;
// The update of one time level that also reduces that level's Eq. (7) sums:
// one DiagPartial per block (update_blocks of them) and, if fields is given,
// u, v, w, mu into fields.
uint32_t update_blocks(const Geom& g, const Launch& lc);
hipError_t launch_update_diag(int storage, void* pop, const Geom& g, const Phys& ph, const Codec& cd, int parity,
                              const Launch& lc, const PhysD& phd, DiagPartial* partials, double* fields,
                              hipStream_t s);
hipError_t launch_diag_sums(int storage, const void* pop, const Geom& g, const Phys& ph, const PhysD& phd,
                            const Codec& cd, int parity, DiagPartial* partials, double* fields, hipStream_t s);
// u, v, w of a periodic lattice into fields (3 * ncells doubles), in the
// arithmetic of launch_diag_sums, reading only the rho and rho u populations.
hipError_t launch_velocity(int storage, const void* pop, const Geom& g, const Codec& cd, int parity, double* fields,
                           hipStream_t s);
// fields: u, v, w, mu (4 * ncells doubles), then div, wx, wy, wz (4 * ncells).
// Spectral eps sums of the u, v, w, mu fields into DIAG_BLOCKS partials: only
// their eps fields, or (full) whole partials with the other fields neutral.
hipError_t launch_spectral(const Geom& g, double dx, double* fields, DiagPartial* partials, bool full,
                           hipStream_t s);
hipError_t launch_diag_final(DiagPartial* partials, int nparts, DiagPartial* out, hipStream_t s);
// The same total in two levels when there are many partials: chunks reduced
// into tmp (at most ntmp of them) by many blocks, then tmp by one block.
hipError_t launch_diag_final2(DiagPartial* partials, int nparts, DiagPartial* tmp, int ntmp, DiagPartial* out,
                              hipStream_t s);
// Shell spectrum of the velocity held in fields (u, v, w: the first 3 * ncells
// doubles, written by launch_diag_sums); uses fields[4 ncells, 7 ncells) as
// workspace and partial (nz * spectrum_shells(nx) doubles).  Writes nout
// values to E (zero beyond the shell count).  Cubic periodic lattices only.
uint32_t spectrum_shells(uint32_t n);
hipError_t launch_spectrum(const Geom& g, double* fields, double* partial, double* E, uint32_t nout, hipStream_t s);

}  // namespace cnsf
