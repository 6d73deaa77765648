/*
 * cnsf.h - C ABI of the D3Q7 compressible Navier-Stokes-Fourier lattice
 * Boltzmann hot path for MI355X (gfx950).
 *
 * The method: the fourteen-component state Q = (rho, rho u, E, tau, q) of
 * Eq. (2) (Section 2.1), one set of seven D3Q7 populations per component with
 * a linear equilibrium embedding the flux in its first moment, zeroth-moment
 * recovery and BGK collide-and-stream with the source on the lattice weights
 * (Section 2.2), the relaxation rate lowered per cell by the local one-sided
 * shock sensor of Eqs. (3)-(6) (Section 2.3), and the volume averages of
 * Eq. (7) (Section 3.2).
 *
 * Conventions for every call:
 *  - Component order k: 0 rho, 1-3 rho*u_{x,y,z}, 4 E, 5-10 tau_{xx,yy,zz,xy,xz,yz},
 *    11-13 q_{x,y,z}.  tau is the Newtonian-sign stress of Eq. (2).
 *  - Field arrays are FP64, component-major, x fastest: Q[k][z][y][x].
 *  - Pointers marked "host or device" are read or written according to the
 *    `where` argument (CNSF_HOST or CNSF_DEVICE); device pointers must be on
 *    the device that was current at cnsf_create.
 *  - Every call returns CNSF_OK or an error code; cnsf_last_error() gives the
 *    message of the last failing call on the calling thread.  No C++
 *    exception crosses this interface.
 *  - Work is enqueued on the HIP stream given at creation.  Calls that return
 *    data to the host synchronise that stream.
 */
#ifndef CNSF_H
#define CNSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CNSF_NCOMP 14
#define CNSF_NVEL 7
#define CNSF_NPOP 98
#define CNSF_ABI_VERSION 1

enum cnsf_status {
  CNSF_OK = 0,
  CNSF_E_INVALID = 1, /* a parameter or argument is out of range */
  CNSF_E_NOMEM = 2,   /* a buffer is too small or an allocation failed */
  CNSF_E_DEVICE = 3,  /* a HIP call failed */
  CNSF_E_STATE = 4,   /* a field holds rho <= 0, p <= 0 or a non-finite value */
  CNSF_E_SIZE = 5     /* mismatched sizes (checkpoint, slab range) */
};

enum cnsf_visc_law { CNSF_VISC_CONST = 0, CNSF_VISC_SUTHERLAND = 1, CNSF_VISC_POWER = 2 };
enum cnsf_bc { CNSF_BC_PERIODIC = 0, CNSF_BC_WALL = 1, CNSF_BC_DIRICHLET = 2, CNSF_BC_NOSLIP = 3 };
enum cnsf_storage { CNSF_STORAGE_FP32 = 0, CNSF_STORAGE_FP16 = 1, CNSF_STORAGE_BF16 = 2 };
enum cnsf_where { CNSF_HOST = 0, CNSF_DEVICE = 1 };

/*
 * Parameters of one lattice (Table "Parameters" of Section 2.3 and the
 * declaration listing of Section 2.1).  Physical units throughout.
 *  size            sizeof(cnsf_params); set by cnsf_params_default.
 *  nx, ny, nz      lattice cells (>= 1 each).  One component's 7 population
 *                  slots are addressed with 32-bit byte offsets, so
 *                  nx*ny*nz <= 153,391,104 for FP32 (535^3) and
 *                  <= 306,783,232 for FP16 / BF16 (674^3).
 *  dx, dt          cell size and time step (> 0); lambda = dx/dt.
 *  gamma           adiabatic index (> 1).
 *  mu0, T_ref      reference viscosity (>= 0) and temperature (> 0).
 *  visc_law        mu_T(T): CONST mu0; SUTHERLAND mu0 (1+S) th^1.5/(th+S) with
 *                  S = visc_param and th = T/T_ref; POWER mu0 th^visc_param.
 *  prandtl         kappa = gamma mu0 / ((gamma-1) Pr) (> 0).
 *  tau_R, tau_q    relaxation times of tau and q (> 0).
 *  f_mu            background dissipation of Eq. (6): tau_base = 1/2 +
 *                  4 f_mu (mu_T/rho) dt/dx^2, evaluated per cell (>= 0).
 *  tau_base_override  if > 0, a constant tau_base (in time steps) instead.
 *  C_sigma, J_min, omega_min  sensor slope, threshold and rate floor of
 *                  Eqs. (3)-(5); C_sigma = 0 disables the sensor.
 *  bc_x            x-ends: PERIODIC; WALL (halfway bounce-back with the mirror
 *                  sign of each component: a slip, adiabatic symmetry plane);
 *                  DIRICHLET (incoming populations set to the equilibrium of
 *                  Q_left / Q_right); NOSLIP (halfway no-slip walls generated
 *                  from the fluxes of Eq. (2): the momentum takes the wall's
 *                  velocity and, on an adiabatic wall, q_x is zero, both by
 *                  anti-bounce-back; every other component returns with its
 *                  Eq. (2) normal flux at the wall state, by bounce-back).
 *                  y and z periodic.
 *  Q_left, Q_right uniform 14-vectors for DIRICHLET.
 *  storage         population storage: FP32, or FP16 / BF16 deviations.
 *  Q_ref           reference state of the shifted storage: populations are
 *                  stored as g = (f - f^eq(Q_ref)) / s_k.
 *  storage_scale   s_k per component (power of two recommended); 0 means 1.
 *  a_ref           optional largest characteristic speed; if > 0, creation
 *                  rejects a_ref dt/dx > 1/2 (sub-characteristic bound).
 *  wall_u[s]       NOSLIP: velocity of the wall at x = 0 (s = 0) and at
 *                  x = nx*dx (s = 1); tangential, so wall_u[s][0] must be 0.
 *  wall_T[s]       NOSLIP: wall temperature (> 0, isothermal) or 0 (adiabatic).
 */
typedef struct cnsf_params {
  uint32_t size;
  int32_t nx, ny, nz;
  double dx, dt;
  double gamma, mu0, T_ref;
  int32_t visc_law;
  double visc_param;
  double prandtl;
  double tau_R, tau_q;
  double f_mu, tau_base_override;
  double C_sigma, J_min, omega_min;
  int32_t bc_x;
  double Q_left[CNSF_NCOMP];
  double Q_right[CNSF_NCOMP];
  int32_t storage;
  double Q_ref[CNSF_NCOMP];
  double storage_scale[CNSF_NCOMP];
  double a_ref;
  double wall_u[2][3];
  double wall_T[2];
} cnsf_params;

/* Volume diagnostics (FP64 reductions on the device).  E_k, eps_s, eps_d follow
 * Eq. (7) with rho_ref = 1 and mu_local from the lattice's viscosity law;
 * eps_s / eps_d use spectral derivatives along each periodic axis (zero when
 * not requested or when bc_x is not periodic). */
typedef struct cnsf_diag {
  int64_t step;
  double time;
  double mass, momentum[3], energy; /* sums over cells of rho, rho u, E */
  double E_k;                       /* <rho |u|^2 / 2> */
  double eps_s, eps_d;              /* <mu |curl u|^2>, 4/3 <mu (div u)^2> */
  double min_rho, min_p;
  double sensor_fraction;           /* fraction of cells with chi > 0 */
  int64_t nonfinite;                /* cells with a non-finite moment */
} cnsf_diag;

enum cnsf_diag_flags { CNSF_DIAG_SUMS = 0, CNSF_DIAG_SPECTRAL = 1 };

typedef struct cnsf_lattice cnsf_lattice;

/* Fill *p with defaults: gamma 1.4, constant viscosity 0, Pr 0.71, sensor
 * off, periodic, FP32 storage, zero reference state.  Never fails for p != NULL. */
int cnsf_params_default(cnsf_params* p);

/* Device bytes of the population array for p: 14 component regions, each
 * holding the 7 slots of every cell (cells in groups of 1024, the 7 slots of a
 * group back to back), 4 bytes (FP32) or 2 bytes (FP16 / BF16) per population,
 * with the cell count rounded up to whole groups.
 * The array is the only large allocation; the in-place (AA) streaming needs
 * no second copy. */
int cnsf_required_bytes(const cnsf_params* p, size_t* bytes);

/* Validate p, derive the lattice constants and bind the population array.
 *  dev_buf  caller-owned device buffer of at least cnsf_required_bytes bytes,
 *           256-byte aligned; never freed by the library.  NULL: the library
 *           allocates (hipMalloc) and frees it in cnsf_destroy.
 *  stream   hipStream_t on which all work is enqueued (NULL: default stream).
 * The whole array is cleared on the stream (the unused slots past the last
 * cell too, so exported checkpoints of equal states are byte-identical).
 * Errors: CNSF_E_INVALID (any range listed under cnsf_params, omega outside
 * (0,2), unknown enum, sub-characteristic bound), CNSF_E_NOMEM, CNSF_E_DEVICE. */
int cnsf_create(const cnsf_params* p, void* dev_buf, size_t bytes, void* stream, cnsf_lattice** out);

/* Release library-owned device memory and the handle. */
int cnsf_destroy(cnsf_lattice* lat);

/* Set the populations of z-planes [z0, z0+nzs) to f^eq(Q) (Section 2.2
 * initial state).  Q (host or device) is [14][nzs][ny][nx].  Resets the
 * step counter (and the parity) when z0 == 0.  The populations are written in
 * the layout of an even time level, so a lattice at an odd level (after an
 * odd number of steps) accepts only a write of the whole lattice, z0 == 0 and
 * nzs == nz; a slab there returns CNSF_E_INVALID and changes nothing (step
 * once more, or write every plane in one call).  CNSF_E_STATE if a cell has
 * rho <= 0, p <= 0 or a non-finite value (checked on the device). */
int cnsf_set_state(cnsf_lattice* lat, const double* Q, int32_t z0, int32_t nzs, int32_t where);

/* As cnsf_set_state, from primitive fields: P (host or device) is
 * [14][nzs][ny][nx] holding rho, u_x, u_y, u_z, p, tau_{xx,yy,zz,xy,xz,yz},
 * q_{x,y,z}; the conserved state (rho, rho u, E = p/(gamma-1) + rho|u|^2/2,
 * tau, q; Section 2.1) is formed on the device in FP64. */
int cnsf_set_primitive(cnsf_lattice* lat, const double* P, int32_t z0, int32_t nzs, int32_t where);

/* Enqueue n fused stream-and-collide updates (Section 2.2, with the sensor of
 * Section 2.3; alternating even/odd in-place passes).  Asynchronous; n >= 0.
 * Lattices of at most 2^21 cells replay a HIP graph of 32 updates, captured on
 * first use, when n >= 64 (the results are those of single launches); while the
 * lattice's stream is itself being captured, the updates are plain launches.
 * CNSF_E_DEVICE if a launch fails. */
int cnsf_step(cnsf_lattice* lat, int64_t n);

/* Time the update on this lattice's population array: one untimed update, then
 * `steps` >= 1 timed ones (HIP events on the lattice's stream); *ms receives
 * their mean time per update.  Synchronises the stream and advances the
 * lattice by 1 + steps.  The same update runs at different speeds in
 * different physical allocations of the array, and an allocation keeps its
 * speed; an allocation policy probes candidate arrays with this and keeps the
 * fastest.  Errors as cnsf_step. */
int cnsf_probe_update_ms(cnsf_lattice* lat, int32_t steps, double* ms);

/* Q_k = sum_i f_{k,i} (the zeroth moment, Section 2.2) of the current time
 * level for z-planes [z0, z0+nzs), written FP64 to out (host or device) as
 * [14][nzs][ny][nx].  CNSF_E_SIZE if the slab leaves the lattice. */
int cnsf_get_moments(cnsf_lattice* lat, double* out, int32_t z0, int32_t nzs, int32_t where);

/* Primitive fields of the current time level for z-planes [z0, z0+nzs),
 * written FP64 to out (host or device) as [6][nzs][ny][nx]: rho, u_x, u_y,
 * u_z, p = (gamma-1)(E - rho|u|^2/2), T = p/rho (Section 2.1).
 * CNSF_E_SIZE if the slab leaves the lattice. */
int cnsf_get_primitives(cnsf_lattice* lat, double* out, int32_t z0, int32_t nzs, int32_t where);

/* FP64 diagnostics of the current time level; flags: CNSF_DIAG_SUMS or
 * CNSF_DIAG_SPECTRAL (adds eps_s, eps_d; allocates eight FP64 cell fields on
 * first use, kept until cnsf_destroy). */
int cnsf_diagnostics(cnsf_lattice* lat, int32_t flags, cnsf_diag* out);

/* Shell-averaged velocity spectrum of the current time level (the spectra of
 * Section 3.2): E[k] = 1/2 sum over wavevectors with nint(|kappa|) = k of
 * sum_c |u_hat_c(kappa)|^2, u = rho u / rho, u_hat the discrete Fourier
 * transform divided by the cell count, kappa integer on the cubic periodic
 * box; every mode is counted, so sum_k E[k] = <|u|^2>/2.  FP64 throughout;
 * the shell sums are taken in a fixed order (bitwise reproducible).
 * cnsf_spectrum_shells gives the shell count 1 + nint(sqrt(3) * (n / 2)).
 * E (host or device) holds nshells >= that count values; entries beyond it
 * are zero.  Uses the spectral workspace of cnsf_diagnostics (allocated on
 * first use) and nz * shells doubles more.  CNSF_E_INVALID unless nx = ny =
 * nz with bc_x = PERIODIC; CNSF_E_SIZE if nshells is too small. */
int cnsf_spectrum_shells(const cnsf_lattice* lat, int32_t* nshells);
int cnsf_spectrum(cnsf_lattice* lat, double* E, int32_t nshells, int32_t where);

/* Advance n >= 1 steps and return the FP64 diagnostics of the time level at
 * entry, the values cnsf_diagnostics(lat, flags, out) would have returned
 * before the call (sums to rounding order; minima and counts exactly).  The
 * first update reads that level anyway: it also forms the sums and writes the
 * velocity fields the spectral derivatives need, so the populations are read
 * once instead of twice.  Returns when the n steps are done (synchronises the
 * stream).  Errors as cnsf_step and cnsf_diagnostics. */
int cnsf_step_diagnostics(cnsf_lattice* lat, int64_t n, int32_t flags, cnsf_diag* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * cnsf_step_diagnostics(lat, n, CNSF_DIAG_SUMS, out), with the per-block partial
 * sums and the final result in a fixed library workspace of
 * CNSF_STATIC_DIAG_PARTIALS + 1 partials (96 bytes each, about 0.8 MB) per GPU,
 * held until the process ends, instead of lattice-owned memory.  Allocates
 * nothing (no hipMalloc, no allocating library call); eps_s and eps_d are
 * zero, as with CNSF_DIAG_SUMS.  The update that reduces the level at entry
 * runs on at most CNSF_STATIC_DIAG_PARTIALS blocks (a persistent grid when the
 * lattice's launch has more tiles); the populations are those of n plain steps
 * and the sums agree with cnsf_step_diagnostics to rounding order (minima and
 * counts exactly).  Every call on one GPU shares that GPU's workspace: calls
 * that overlap on one GPU (from several host threads or streams) race and
 * must be serialised by the caller.  Errors: CNSF_E_INVALID (NULL argument,
 * n < 1), CNSF_E_SIZE if cnsf_set_launch set a persistent grid of more than
 * CNSF_STATIC_DIAG_PARTIALS blocks, CNSF_E_DEVICE. */
#define CNSF_STATIC_DIAG_PARTIALS 8192
int cnsf_step_diagnostics_static(cnsf_lattice* lat, int64_t n, cnsf_diag* out);

/* Step counter, parity and the byte size of an exported checkpoint. */
int cnsf_get_info(const cnsf_lattice* lat, int64_t* step, int32_t* parity, size_t* checkpoint_bytes);

/* Copy the raw stored populations (device -> host) with the parity and step;
 * host buffer of checkpoint_bytes.  Import restores them into a lattice made
 * from the same parameters (CNSF_E_SIZE otherwise). */
int cnsf_export_populations(cnsf_lattice* lat, void* host, size_t bytes, int64_t* step, int32_t* parity);
int cnsf_import_populations(cnsf_lattice* lat, const void* host, size_t bytes, int64_t step, int32_t parity);

/* Plain device-to-device copy kernel of `bytes` (multiple of 16), used to
 * measure the attainable HBM bandwidth next to the update. */
int cnsf_hbm_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Kernel launch shape of the update.  Each block owns a tile of `tile`
 * consecutive cells (a multiple of `block`) and walks it `block` cells at a
 * time; grid = 0 launches one block per tile, grid > 0 a persistent grid of
 * that many blocks striding over the tiles; xcd_remap gives each of the 8 XCDs
 * one contiguous span of tiles.  block: 64..256 in steps of 64 (the kernels are
 * compiled for at most 256).  Defaults are the shapes measured fastest on
 * MI355X for the lattice's storage type. */
int cnsf_set_launch(cnsf_lattice* lat, int32_t block, int32_t tile, int32_t grid, int32_t xcd_remap);
int cnsf_get_launch(const cnsf_lattice* lat, int32_t* block, int32_t* tile, int32_t* grid, int32_t* xcd_remap);

const char* cnsf_last_error(void);
const char* cnsf_status_string(int status);

/* ------------------------------------------------------------------------
 * Batched ensembles: many independent lattices (own size, parameters and
 * populations) advanced by one launch per step over a descriptor table, the
 * steps replayed from a captured HIP graph.  All members share the storage
 * type and bc_x = PERIODIC.
 */
typedef struct cnsf_batch cnsf_batch;

/* Create a batch of n members (1 <= n <= 65536).  dev_buf / bytes as in cnsf_create (cleared the
 * same way), at least cnsf_batch_required_bytes (NULL: library-allocated, exactly that size).
 * Layout: when the members' populations of one component (7 slots each) sum to less than 4 GiB,
 * component k of every member forms one run and the 14 runs are spaced evenly; a caller buffer
 * larger than required spreads the runs further apart (spacing = bytes / 14, at most 4 GiB),
 * which the update runs faster on MI355X (about a gigabyte apart, as in a 512^3 lattice).
 * Results do not depend on the layout.  Otherwise members are stored one after another. */
int cnsf_batch_required_bytes(const cnsf_params* members, int32_t n, size_t* bytes);
int cnsf_batch_create(const cnsf_params* members, int32_t n, void* dev_buf, size_t bytes, void* stream,
                      cnsf_batch** out);
int cnsf_batch_destroy(cnsf_batch* b);
/* Member j's initial state (as cnsf_set_state, whole lattice). */
int cnsf_batch_set_state(cnsf_batch* b, int32_t j, const double* Q, int32_t where);
/* Advance every member by n steps.  mode 0: one launch per step over all
 * members; mode 1: the same launches replayed from a HIP graph of
 * `graph_steps` steps (captured on first use); mode 2: one launch per member
 * per step (the sequential baseline). */
int cnsf_batch_step(cnsf_batch* b, int64_t n, int32_t mode);
/* Member j's moments (as cnsf_get_moments, whole lattice). */
int cnsf_batch_get_moments(cnsf_batch* b, int32_t j, double* out, int32_t where);
/* Launch shape of the batched kernel: threads per block (64..256, multiple of
 * 64), cells per tile (multiple of block), persistent grid size in blocks
 * (0: one block per tile), and the number of steps captured per graph. */
int cnsf_batch_set_launch(cnsf_batch* b, int32_t block, int32_t tile, int32_t grid, int32_t graph_steps);
/* The batch's current launch shape (any output pointer may be NULL). */
int cnsf_batch_get_launch(const cnsf_batch* b, int32_t* block, int32_t* tile, int32_t* grid, int32_t* graph_steps);
/* Time candidate launch shapes with HIP events and keep the fastest; results
 * are cached in the JSON file `cache_path` (may be NULL) keyed by the batch's
 * shape signature. */
int cnsf_batch_autotune(cnsf_batch* b, const char* cache_path, int32_t steps_per_trial);

#ifdef __cplusplus
}
#endif

#endif /* CNSF_H */
