// C ABI of the cnsf library: parameter validation, derived lattice constants,
// lattice lifecycle, state set/readout, stepping, diagnostics, checkpoints.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cnsf.h"
#include "api_common.h"
#include "cnsf_impl.h"
#include "launch.h"

using namespace cnsf;

namespace cnsf {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(CNSF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

size_t elem_bytes(int storage) { return storage == CNSF_STORAGE_FP32 ? 4 : 2; }

int validate(const cnsf_params* p) {
  if (!p) return fail(CNSF_E_INVALID, "params is NULL");
  if (p->size != sizeof(cnsf_params))
    return fail(CNSF_E_INVALID, "params.size %u != %zu (use cnsf_params_default)", p->size, sizeof(cnsf_params));
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(CNSF_E_INVALID, "grid %d x %d x %d", p->nx, p->ny, p->nz);
  const uint64_t nc = (uint64_t)p->nx * p->ny * p->nz;
  if (nc >= (1ull << 31)) return fail(CNSF_E_INVALID, "%llu cells exceed 2^31 - 1", (unsigned long long)nc);
  auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
  if (!pos(p->dx) || !pos(p->dt)) return fail(CNSF_E_INVALID, "dx = %g, dt = %g must be > 0", p->dx, p->dt);
  if (!(std::isfinite(p->gamma) && p->gamma > 1.0)) return fail(CNSF_E_INVALID, "gamma = %g must be > 1", p->gamma);
  if (!(std::isfinite(p->mu0) && p->mu0 >= 0.0)) return fail(CNSF_E_INVALID, "mu0 = %g must be >= 0", p->mu0);
  if (!pos(p->T_ref)) return fail(CNSF_E_INVALID, "T_ref = %g must be > 0", p->T_ref);
  if (p->visc_law < 0 || p->visc_law > 2) return fail(CNSF_E_INVALID, "visc_law %d unknown", p->visc_law);
  if (p->visc_law == CNSF_VISC_SUTHERLAND && !pos(p->visc_param))
    return fail(CNSF_E_INVALID, "Sutherland constant %g must be > 0", p->visc_param);
  if (!pos(p->prandtl)) return fail(CNSF_E_INVALID, "prandtl = %g must be > 0", p->prandtl);
  if (!pos(p->tau_R) || !pos(p->tau_q)) return fail(CNSF_E_INVALID, "tau_R, tau_q must be > 0");
  if (!(std::isfinite(p->f_mu) && p->f_mu >= 0.0)) return fail(CNSF_E_INVALID, "f_mu = %g must be >= 0", p->f_mu);
  if (!std::isfinite(p->tau_base_override) || (p->tau_base_override > 0.0 && p->tau_base_override < 0.5))
    return fail(CNSF_E_INVALID, "tau_base_override = %g gives omega outside (0, 2]", p->tau_base_override);
  if (!(std::isfinite(p->C_sigma) && p->C_sigma >= 0.0) || !(std::isfinite(p->J_min) && p->J_min >= 0.0))
    return fail(CNSF_E_INVALID, "C_sigma, J_min must be >= 0");
  if (!(p->omega_min > 0.0 && p->omega_min <= 2.0))
    return fail(CNSF_E_INVALID, "omega_min = %g outside (0, 2]", p->omega_min);
  if (p->C_sigma > 0.0 && p->mu0 <= 0.0) return fail(CNSF_E_INVALID, "the sensor needs mu0 > 0");
  if (p->bc_x < 0 || p->bc_x > 3) return fail(CNSF_E_INVALID, "bc_x %d unknown", p->bc_x);
  if (p->storage < 0 || p->storage > 2) return fail(CNSF_E_INVALID, "storage %d unknown", p->storage);
  for (int k = 0; k < NC; ++k)
    if (!(std::isfinite(p->storage_scale[k]) && p->storage_scale[k] >= 0.0))
      return fail(CNSF_E_INVALID, "storage_scale[%d] = %g", k, p->storage_scale[k]);
  if (p->Q_ref[0] > 0.0) {
    for (int k = 1; k < NC; ++k)
      if (k != 4 && p->Q_ref[k] != 0.0)
        return fail(CNSF_E_INVALID, "Q_ref must be a gas at rest: Q_ref[%d] = %g", k, p->Q_ref[k]);
    if (!((p->gamma - 1.0) * p->Q_ref[4] > 0.0)) return fail(CNSF_E_INVALID, "Q_ref has p <= 0");
  }
  // one component's region is addressed with 32-bit byte offsets
  if (component_stride(nc, p->storage) * elem_bytes(p->storage) >= (1ull << 32) - 256)
    return fail(CNSF_E_INVALID, "%llu cells: one component's 7 population slots exceed 4 GiB", (unsigned long long)nc);
  if (p->a_ref > 0.0 && p->a_ref * p->dt / p->dx > 0.5 * (1.0 + 1e-12))
    return fail(CNSF_E_INVALID, "a_ref dt / dx = %g exceeds the sub-characteristic bound 1/2",
                p->a_ref * p->dt / p->dx);
  if (p->bc_x == CNSF_BC_NOSLIP) {
    for (int s = 0; s < 2; ++s) {
      for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->wall_u[s][a])) return fail(CNSF_E_INVALID, "wall_u[%d][%d] is not finite", s, a);
      if (p->wall_u[s][0] != 0.0)
        return fail(CNSF_E_INVALID, "wall_u[%d][0] = %g: a wall moves tangentially only", s, p->wall_u[s][0]);
      if (!(std::isfinite(p->wall_T[s]) && p->wall_T[s] >= 0.0))
        return fail(CNSF_E_INVALID, "wall_T[%d] = %g must be > 0 (isothermal) or 0 (adiabatic)", s, p->wall_T[s]);
    }
  }
  if (p->bc_x == CNSF_BC_DIRICHLET) {
    for (const double* Qe : {p->Q_left, p->Q_right}) {
      const double rho = Qe[0];
      if (!(rho > 0.0)) return fail(CNSF_E_INVALID, "Dirichlet end state has rho <= 0");
      const double ke = 0.5 * (Qe[1] * Qe[1] + Qe[2] * Qe[2] + Qe[3] * Qe[3]) / rho;
      if (!((p->gamma - 1.0) * (Qe[4] - ke) > 0.0)) return fail(CNSF_E_INVALID, "Dirichlet end state has p <= 0");
    }
  }
  return CNSF_OK;
}

PhysD derive_phys_d(const cnsf_params* p) {
  PhysD d{};
  d.four_over_lam = 4.0 * p->dt / p->dx;
  d.dt = p->dt;
  d.gm1 = p->gamma - 1.0;
  d.mu0 = p->mu0;
  d.inv_Tref = 1.0 / p->T_ref;
  d.visc_param = p->visc_param;
  d.visc_law = p->visc_law;
  d.inv_tauR = 1.0 / p->tau_R;
  d.inv_tauq = 1.0 / p->tau_q;
  // K_q = kappa (mu_T / mu0) / tau_q with kappa = gamma mu0 / ((gamma - 1) Pr)
  d.kq_over_mu0 = p->gamma / ((p->gamma - 1.0) * p->prandtl * p->tau_q);
  d.three_tauR_4 = 0.75 * p->tau_R;
  d.fmu_coef = 4.0 * p->f_mu * p->dt / (p->dx * p->dx);
  d.tb_override = p->tau_base_override > 0.0 ? p->tau_base_override : 0.0;
  d.C_sigma = p->C_sigma;
  d.J_min = p->J_min;
  d.omega_min = p->omega_min;
  return d;
}

Phys to_float(const PhysD& d) {
  Phys f{};
  f.four_over_lam = (float)d.four_over_lam;
  f.dt = (float)d.dt;
  f.gm1 = (float)d.gm1;
  f.mu0 = (float)d.mu0;
  f.inv_Tref = (float)d.inv_Tref;
  f.visc_param = (float)d.visc_param;
  f.visc_law = d.visc_law;
  f.inv_tauR = (float)d.inv_tauR;
  f.inv_tauq = (float)d.inv_tauq;
  f.kq_over_mu0 = (float)d.kq_over_mu0;
  f.three_tauR_4 = (float)d.three_tauR_4;
  f.fmu_coef = (float)d.fmu_coef;
  f.tb_override = (float)d.tb_override;
  f.C_sigma = (float)d.C_sigma;
  f.J_min = (float)d.J_min;
  f.omega_min = (float)d.omega_min;
  return f;
}

// FP64 equilibrium of a uniform 14-vector (host side).
void uniform_feq(const double* Qv, const PhysD& ph, double feq[NC][NV]) {
  double Q[NC];
  for (int k = 0; k < NC; ++k) Q[k] = Qv[k];
  Prim<double> P = primitives<double>(Q, ph);
  equilibrium_all<double>(Q, P, ph.four_over_lam, feq);
}

Codec derive_codec(const cnsf_params* p, const PhysD& ph) {
  Codec cd{};
  if (p->Q_ref[0] > 0.0) {
    double f[NC][NV];
    uniform_feq(p->Q_ref, ph, f);
    cd.rho_w = (float)p->Q_ref[0];
    cd.E_w = (float)p->Q_ref[4];
    cd.fm = (float)f[1][1];    // w_1 (4/lambda) p_ref
    cd.fq = (float)f[11][1];   // w_1 (4/lambda) (K_q T)_ref
    cd.KT_ref = (float)(f[11][1] / (0.125 * ph.four_over_lam));
  }
  for (int k = 0; k < NC; ++k) {
    const double s = p->storage_scale[k] > 0.0 ? p->storage_scale[k] : 1.0;
    cd.scale[k] = (float)s;
    cd.inv_scale[k] = (float)(1.0 / s);
    if (s != 1.0 && p->storage != CNSF_STORAGE_FP32) cd.scaled = 1;
  }
  return cd;
}

Geom derive_geom(const cnsf_params* p, const PhysD& ph) {
  Geom g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.nxy = (uint32_t)p->nx * p->ny;
  g.ncells = g.nxy * (uint32_t)p->nz;
  g.cstride = component_stride(g.ncells, p->storage);
  g.bc_x = p->bc_x;
  if (p->bc_x == CNSF_BC_DIRICHLET) {
    const Codec cd = derive_codec(p, ph);
    double fl[NC][NV], fr[NC][NV];
    uniform_feq(p->Q_left, ph, fl);
    uniform_feq(p->Q_right, ph, fr);
    for (int k = 0; k < NC; ++k) {
      g.dev_left[k] = (float)(fl[k][1] - feq_ref<double>(cd, k, 1));
      g.dev_right[k] = (float)(fr[k][2] - feq_ref<double>(cd, k, 2));
    }
  }
  if (p->bc_x == CNSF_BC_NOSLIP) {
    const Codec cd = derive_codec(p, ph);
    for (int s = 0; s < 2; ++s) {
      const double Tw = p->wall_T[s];
      g.wall_uy[s] = (float)p->wall_u[s][1];
      g.wall_uz[s] = (float)p->wall_u[s][2];
      g.wall_iso[s] = Tw > 0.0 ? 1 : 0;
      if (Tw > 0.0) {
        const double mu = mu_of_T<double>(Tw, ph);
        g.wall_nuR[s] = (float)(mu * ph.inv_tauR);
        g.wall_dKT[s] = (float)(ph.kq_over_mu0 * mu * Tw - (double)cd.KT_ref);
      }
    }
  }
  return g;
}

}  // namespace cnsf

constexpr int STEP_FINAL_CHUNKS = 1024;   // chunk sums of the fused diagnostic step's final reduction

struct cnsf_lattice {
  cnsf_params p;
  Geom g;
  Phys ph;
  PhysD phd;
  Codec cd;
  void* pop = nullptr;
  bool owned = false;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t step = 0;
  int parity = 0;
  Launch lc;
  int* dflag = nullptr;               // device error flag
  DiagPartial* partials = nullptr;    // diagnostics block partials
  DiagPartial* dresult = nullptr;
  double* fields = nullptr;           // spectral workspace (8 doubles per cell)
  double* spec = nullptr;             // shell-spectrum partials and output
  DiagPartial* step_partials = nullptr;  // per-block sums of the fused diagnostic step
  uint32_t step_partials_cap = 0;
  DiagPartial* dresult2 = nullptr;       // eps sums of the fused diagnostic step
  // small lattices: GRAPH_STEPS updates captured once and replayed (launch-bound otherwise)
  hipStream_t gstream = nullptr;         // capture stream
  hipGraphExec_t gexec = nullptr;
};

namespace {
// Lattices up to this many cells step through a replayed HIP graph when a call
// asks for at least 2 GRAPH_STEPS updates: their update takes a few
// microseconds, about what one launch costs.  Larger lattices launch directly.
constexpr uint32_t GRAPH_MAX_CELLS = 1u << 21;
constexpr int64_t GRAPH_STEPS = 32;   // even: a replay starts and ends at even parity

void drop_graph(cnsf_lattice* L) {
  if (L->gexec) (void)hipGraphExecDestroy(L->gexec);
  L->gexec = nullptr;
}

hipError_t launch_steps(cnsf_lattice* L, int64_t n, hipStream_t s, int& parity) {
  for (int64_t i = 0; i < n; ++i) {
    hipError_t e = launch_update(L->p.storage, L->pop, L->g, L->ph, L->cd, parity, L->lc, s);
    if (e != hipSuccess) return e;
    parity ^= 1;
  }
  return hipSuccess;
}

// GRAPH_STEPS updates from even parity, captured on the lattice's own capture
// stream (the caller's stream may be the null stream, which cannot capture).
hipError_t build_graph(cnsf_lattice* L) {
  hipError_t e = hipSuccess;
  if (!L->gstream) e = hipStreamCreateWithFlags(&L->gstream, hipStreamNonBlocking);
  hipGraph_t graph = nullptr;
  if (e == hipSuccess) e = hipStreamBeginCapture(L->gstream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    int par = 0;
    hipError_t el = launch_steps(L, GRAPH_STEPS, L->gstream, par);
    e = hipStreamEndCapture(L->gstream, &graph);
    if (el != hipSuccess) e = el;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&L->gexec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}
}  // namespace

extern "C" {

int cnsf_params_default(cnsf_params* p) {
  if (!p) return fail(CNSF_E_INVALID, "params is NULL");
  std::memset(p, 0, sizeof *p);
  p->size = sizeof *p;
  p->nx = p->ny = p->nz = 1;
  p->dx = 1.0;
  p->dt = 0.1;
  p->gamma = 1.4;
  p->mu0 = 0.0;
  p->T_ref = 1.0;
  p->visc_law = CNSF_VISC_CONST;
  p->prandtl = 0.71;
  p->tau_R = p->tau_q = 1.0;
  p->omega_min = 1.0;
  p->bc_x = CNSF_BC_PERIODIC;
  p->storage = CNSF_STORAGE_FP32;
  return CNSF_OK;
}

int cnsf_required_bytes(const cnsf_params* p, size_t* bytes) {
  if (int e = validate(p)) return e;
  if (!bytes) return fail(CNSF_E_INVALID, "bytes is NULL");
  const uint64_t nc = (uint64_t)p->nx * p->ny * p->nz;
  *bytes = (size_t)NC * component_stride(nc, p->storage) * elem_bytes(p->storage);
  return CNSF_OK;
}

int cnsf_create(const cnsf_params* p, void* dev_buf, size_t bytes, void* stream, cnsf_lattice** out) {
  if (!out) return fail(CNSF_E_INVALID, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  if (int e = cnsf_required_bytes(p, &need)) return e;
  if (dev_buf && bytes < need) return fail(CNSF_E_NOMEM, "buffer of %zu bytes < required %zu", bytes, need);
  if (dev_buf && ((uintptr_t)dev_buf & 255u)) return fail(CNSF_E_INVALID, "buffer not 256-byte aligned");
  auto* L = new cnsf_lattice();
  L->p = *p;
  L->phd = derive_phys_d(p);
  L->ph = to_float(L->phd);
  L->g = derive_geom(p, L->phd);
  L->cd = derive_codec(p, L->phd);
  L->stream = (hipStream_t)stream;
  L->bytes = need;
  L->lc = default_launch(p->storage);
  (void)hipGetDevice(&L->device);
  hipError_t e;
  if (dev_buf) {
    L->pop = dev_buf;
  } else {
    e = hipMalloc(&L->pop, need);
    if (e != hipSuccess) {
      delete L;
      return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    }
    L->owned = true;
  }
  e = hipMalloc(&L->dflag, sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&L->partials, sizeof(DiagPartial) * (DIAG_BLOCKS + 1));
  if (e == hipSuccess) e = hipMalloc(&L->dresult, sizeof(DiagPartial));
  if (e != hipSuccess) {
    cnsf_destroy(L);
    return fail(CNSF_E_NOMEM, "hipMalloc of small buffers: %s", hipGetErrorString(e));
  }
  // the slots past the last cell of the final group are never written by a
  // step; cleared here, equal states export byte-identical checkpoints
  e = hipMemsetAsync(L->pop, 0, need, L->stream);
  if (e != hipSuccess) {
    cnsf_destroy(L);
    return hip_fail(e, "clearing the population array");
  }
  *out = L;
  return CNSF_OK;
}

int cnsf_destroy(cnsf_lattice* L) {
  if (!L) return CNSF_OK;
  (void)hipSetDevice(L->device);
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  else (void)hipDeviceSynchronize();
  if (L->owned && L->pop) (void)hipFree(L->pop);
  if (L->dflag) (void)hipFree(L->dflag);
  if (L->partials) (void)hipFree(L->partials);
  if (L->dresult) (void)hipFree(L->dresult);
  if (L->fields) (void)hipFree(L->fields);
  if (L->spec) (void)hipFree(L->spec);
  if (L->step_partials) (void)hipFree(L->step_partials);
  if (L->dresult2) (void)hipFree(L->dresult2);
  drop_graph(L);
  if (L->gstream) (void)hipStreamDestroy(L->gstream);
  delete L;
  return CNSF_OK;
}

int cnsf_set_launch(cnsf_lattice* L, int32_t block, int32_t tile, int32_t grid, int32_t xcd_remap) {
  if (!L) return fail(CNSF_E_INVALID, "lattice is NULL");
  if (block < 64 || block > 256 || block % 64) return fail(CNSF_E_INVALID, "block %d not a multiple of 64 in [64, 256]", block);
  if (tile < block || tile % block) return fail(CNSF_E_INVALID, "tile %d must be a multiple of block %d", tile, block);
  if (grid < 0) return fail(CNSF_E_INVALID, "grid %d < 0", grid);
  L->lc.block = block;
  L->lc.tile = tile;
  L->lc.grid = grid;
  L->lc.remap = xcd_remap ? 1 : 0;
  drop_graph(L);   // the captured updates carry the old shape
  return CNSF_OK;
}

static int set_state_impl(cnsf_lattice* L, const double* Q, int32_t z0, int32_t nzs, int32_t where, bool prim) {
  if (!L || !Q) return fail(CNSF_E_INVALID, "NULL argument");
  if (z0 < 0 || nzs < 0 || z0 + nzs > (int)L->g.nz) return fail(CNSF_E_SIZE, "slab [%d, %d) outside nz = %u", z0, z0 + nzs, L->g.nz);
  if (where != CNSF_HOST && where != CNSF_DEVICE) return fail(CNSF_E_INVALID, "where = %d", where);
  // the initial populations are written in the even-pass layout (slot i of
  // the cell itself); at an odd time level the other planes are stored in the
  // odd layout, so only a write of the whole lattice (which restarts at an
  // even level) keeps the array consistent
  if (L->parity != 0 && !(z0 == 0 && nzs == (int)L->g.nz))
    return fail(CNSF_E_INVALID,
                "lattice at an odd time level (step %lld): set the whole lattice (z0 = 0, nzs = %u) or step once more",
                (long long)L->step, L->g.nz);
  (void)hipSetDevice(L->device);
  const uint32_t nslab = (uint32_t)nzs * L->g.nxy;
  const uint32_t cell0 = (uint32_t)z0 * L->g.nxy;
  const size_t qbytes = (size_t)NC * nslab * sizeof(double);
  const double* dQ = Q;
  double* tmp = nullptr;
  hipError_t e;
  if (where == CNSF_HOST && nslab) {
    e = hipMalloc(&tmp, qbytes);
    if (e != hipSuccess) return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", qbytes, hipGetErrorString(e));
    e = hipMemcpyAsync(tmp, Q, qbytes, hipMemcpyHostToDevice, L->stream);
    if (e != hipSuccess) { (void)hipFree(tmp); return hip_fail(e, "hipMemcpyAsync"); }
    dQ = tmp;
  }
  int bad = 0;
  e = hipMemsetAsync(L->dflag, 0, sizeof(int), L->stream);
  if (e == hipSuccess)
    e = launch_init(L->p.storage, L->pop, dQ, L->g, L->phd, L->cd, cell0, nslab, L->dflag, prim, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, L->dflag, sizeof(int), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "set_state");
  if (z0 == 0) {
    L->step = 0;
    L->parity = 0;
  }
  if (bad) return fail(CNSF_E_STATE, "state has rho <= 0, p <= 0 or a non-finite value in z-planes [%d, %d)", z0, z0 + nzs);
  return CNSF_OK;
}

int cnsf_step(cnsf_lattice* L, int64_t n) {
  if (!L) return fail(CNSF_E_INVALID, "lattice is NULL");
  if (n < 0) return fail(CNSF_E_INVALID, "n = %lld < 0", (long long)n);
  (void)hipSetDevice(L->device);
  int64_t left = n;
  hipError_t e = hipSuccess;
  // a caller that is capturing its own stream gets plain launches in its graph
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (L->stream) (void)hipStreamIsCapturing(L->stream, &cap);
  if (L->g.ncells <= GRAPH_MAX_CELLS && n >= 2 * GRAPH_STEPS && cap == hipStreamCaptureStatusNone) {
    if (L->parity) {
      e = launch_steps(L, 1, L->stream, L->parity);
      --left;
    }
    if (e == hipSuccess && !L->gexec) e = build_graph(L);
    // the replays run on the caller's stream, in its order with its other work
    for (; e == hipSuccess && left >= GRAPH_STEPS; left -= GRAPH_STEPS) e = hipGraphLaunch(L->gexec, L->stream);
  }
  if (e == hipSuccess) e = launch_steps(L, left, L->stream, L->parity);
  if (e != hipSuccess) return hip_fail(e, "update launch");
  L->step += n;
  return CNSF_OK;
}

int cnsf_probe_update_ms(cnsf_lattice* L, int32_t steps, double* ms) {
  if (!L || !ms) return fail(CNSF_E_INVALID, "NULL argument");
  if (steps < 1) return fail(CNSF_E_INVALID, "steps = %d < 1", steps);
  (void)hipSetDevice(L->device);
  if (int r = cnsf_step(L, 1)) return r;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, L->stream);
  int r = CNSF_OK;
  if (e == hipSuccess) r = cnsf_step(L, steps);
  if (e == hipSuccess && r == CNSF_OK) e = hipEventRecord(b, L->stream);
  if (e == hipSuccess && r == CNSF_OK) e = hipEventSynchronize(b);
  float t = 0.0f;
  if (e == hipSuccess && r == CNSF_OK) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (r != CNSF_OK) return r;
  if (e != hipSuccess) return hip_fail(e, "probe timing");
  *ms = (double)t / steps;
  return CNSF_OK;
}

int cnsf_set_state(cnsf_lattice* L, const double* Q, int32_t z0, int32_t nzs, int32_t where) {
  return set_state_impl(L, Q, z0, nzs, where, false);
}

int cnsf_set_primitive(cnsf_lattice* L, const double* P, int32_t z0, int32_t nzs, int32_t where) {
  return set_state_impl(L, P, z0, nzs, where, true);
}

int cnsf_get_primitives(cnsf_lattice* L, double* out, int32_t z0, int32_t nzs, int32_t where) {
  if (!L || !out) return fail(CNSF_E_INVALID, "NULL argument");
  if (z0 < 0 || nzs < 0 || z0 + nzs > (int)L->g.nz) return fail(CNSF_E_SIZE, "slab [%d, %d) outside nz = %u", z0, z0 + nzs, L->g.nz);
  if (where != CNSF_HOST && where != CNSF_DEVICE) return fail(CNSF_E_INVALID, "where = %d", where);
  (void)hipSetDevice(L->device);
  const uint32_t nslab = (uint32_t)nzs * L->g.nxy;
  const uint32_t cell0 = (uint32_t)z0 * L->g.nxy;
  const size_t pbytes = (size_t)6 * nslab * sizeof(double);
  double* dst = out;
  double* tmp = nullptr;
  hipError_t e;
  if (where == CNSF_HOST && nslab) {
    e = hipMalloc(&tmp, pbytes);
    if (e != hipSuccess) return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", pbytes, hipGetErrorString(e));
    dst = tmp;
  }
  e = launch_primitives(L->p.storage, L->pop, dst, L->g, L->cd, L->phd, L->parity, cell0, nslab, L->stream);
  if (e == hipSuccess && tmp) e = hipMemcpyAsync(out, tmp, pbytes, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "get_primitives");
  return CNSF_OK;
}

int cnsf_get_moments(cnsf_lattice* L, double* out, int32_t z0, int32_t nzs, int32_t where) {
  if (!L || !out) return fail(CNSF_E_INVALID, "NULL argument");
  if (z0 < 0 || nzs < 0 || z0 + nzs > (int)L->g.nz) return fail(CNSF_E_SIZE, "slab [%d, %d) outside nz = %u", z0, z0 + nzs, L->g.nz);
  if (where != CNSF_HOST && where != CNSF_DEVICE) return fail(CNSF_E_INVALID, "where = %d", where);
  (void)hipSetDevice(L->device);
  const uint32_t nslab = (uint32_t)nzs * L->g.nxy;
  const uint32_t cell0 = (uint32_t)z0 * L->g.nxy;
  const size_t qbytes = (size_t)NC * nslab * sizeof(double);
  double* dst = out;
  double* tmp = nullptr;
  hipError_t e;
  if (where == CNSF_HOST && nslab) {
    e = hipMalloc(&tmp, qbytes);
    if (e != hipSuccess) return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", qbytes, hipGetErrorString(e));
    dst = tmp;
  }
  e = launch_moments(L->p.storage, L->pop, dst, L->g, L->cd, L->parity, cell0, nslab, L->stream);
  if (e == hipSuccess && tmp) e = hipMemcpyAsync(out, tmp, qbytes, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "get_moments");
  return CNSF_OK;
}

static void fill_diag(const cnsf_lattice* L, const DiagPartial& r, bool spectral, int64_t step, cnsf_diag* d) {
  const double n = (double)L->g.ncells;
  d->step = step;
  d->time = (double)step * L->p.dt;
  d->mass = r.mass;
  d->momentum[0] = r.mx;
  d->momentum[1] = r.my;
  d->momentum[2] = r.mz;
  d->energy = r.energy;
  d->E_k = 0.5 * r.ek2 / n;
  d->eps_s = spectral ? r.eps_s / n : 0.0;
  d->eps_d = spectral ? 4.0 / 3.0 * r.eps_d / n : 0.0;
  d->min_rho = r.min_rho;
  d->min_p = r.min_p;
  d->sensor_fraction = r.sensor / n;
  d->nonfinite = (int64_t)r.nonfinite;
}

int cnsf_diagnostics(cnsf_lattice* L, int32_t flags, cnsf_diag* d) {
  if (!L || !d) return fail(CNSF_E_INVALID, "NULL argument");
  (void)hipSetDevice(L->device);
  const bool spectral = (flags & CNSF_DIAG_SPECTRAL) && L->g.bc_x == CNSF_BC_PERIODIC;
  hipError_t e = hipSuccess;
  if (spectral && !L->fields) {
    e = hipMalloc(&L->fields, (size_t)8 * L->g.ncells * sizeof(double));
    if (e != hipSuccess) {
      L->fields = nullptr;
      return fail(CNSF_E_NOMEM, "spectral workspace: %s", hipGetErrorString(e));
    }
  }
  e = launch_diag_sums(L->p.storage, L->pop, L->g, L->ph, L->phd, L->cd, L->parity, L->partials,
                       spectral ? L->fields : nullptr, L->stream);
  if (e == hipSuccess && spectral) e = launch_spectral(L->g, L->p.dx, L->fields, L->partials, false, L->stream);
  if (e == hipSuccess) e = launch_diag_final(L->partials, DIAG_BLOCKS, L->dresult, L->stream);
  DiagPartial r{};
  if (e == hipSuccess) e = hipMemcpyAsync(&r, L->dresult, sizeof r, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostics");
  fill_diag(L, r, spectral, L->step, d);
  return CNSF_OK;
}

int cnsf_step_diagnostics(cnsf_lattice* L, int64_t n, int32_t flags, cnsf_diag* d) {
  if (!L || !d) return fail(CNSF_E_INVALID, "NULL argument");
  if (n < 1) return fail(CNSF_E_INVALID, "n = %lld < 1", (long long)n);
  (void)hipSetDevice(L->device);
  const bool spectral = (flags & CNSF_DIAG_SPECTRAL) && L->g.bc_x == CNSF_BC_PERIODIC;
  hipError_t e = hipSuccess;
  if (spectral && !L->fields) {
    e = hipMalloc(&L->fields, (size_t)8 * L->g.ncells * sizeof(double));
    if (e != hipSuccess) {
      L->fields = nullptr;
      return fail(CNSF_E_NOMEM, "spectral workspace: %s", hipGetErrorString(e));
    }
  }
  const uint32_t nb = update_blocks(L->g, L->lc);
  if (L->step_partials_cap < nb) {
    if (L->step_partials) (void)hipFree(L->step_partials);
    L->step_partials = nullptr;
    L->step_partials_cap = 0;
    // the block partials, then room for the chunk sums of the two-level final reduction
    e = hipMalloc(&L->step_partials, (size_t)(nb + STEP_FINAL_CHUNKS) * sizeof(DiagPartial));
    if (e != hipSuccess) {
      L->step_partials = nullptr;
      return fail(CNSF_E_NOMEM, "step partials: %s", hipGetErrorString(e));
    }
    L->step_partials_cap = nb;
  }
  if (!L->dresult2) {
    e = hipMalloc(&L->dresult2, sizeof(DiagPartial));
    if (e != hipSuccess) {
      L->dresult2 = nullptr;
      return fail(CNSF_E_NOMEM, "diagnostic result: %s", hipGetErrorString(e));
    }
  }
  const int64_t step0 = L->step;
  // the first update reduces the sums of the level it reads and writes u, v, w, mu
  e = launch_update_diag(L->p.storage, L->pop, L->g, L->ph, L->cd, L->parity, L->lc, L->phd, L->step_partials,
                         spectral ? L->fields : nullptr, L->stream);
  if (e != hipSuccess) return hip_fail(e, "fused diagnostic update");
  L->parity ^= 1;
  ++L->step;
  if (spectral) e = launch_spectral(L->g, L->p.dx, L->fields, L->partials, true, L->stream);
  if (e == hipSuccess)
    e = launch_diag_final2(L->step_partials, (int)nb, L->step_partials + nb, STEP_FINAL_CHUNKS, L->dresult, L->stream);
  if (e == hipSuccess && spectral) e = launch_diag_final(L->partials, DIAG_BLOCKS, L->dresult2, L->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostic reductions");
  if (int r = cnsf_step(L, n - 1)) return r;
  DiagPartial r{}, r2{};
  e = hipMemcpyAsync(&r, L->dresult, sizeof r, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess && spectral) e = hipMemcpyAsync(&r2, L->dresult2, sizeof r2, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "step_diagnostics");
  r.eps_s = r2.eps_s;
  r.eps_d = r2.eps_d;
  fill_diag(L, r, spectral, step0, d);
  return CNSF_OK;
}

}  // extern "C"

// Workspace of cnsf_step_diagnostics_static: the per-block partial sums of
// the first update and, after them, the final result.  One copy per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel: it takes the device address of each GPU's copy once, with
// hipGetSymbolAddress, and uses that.
namespace {
constexpr int STATIC_PARTIALS = CNSF_STATIC_DIAG_PARTIALS;
static __device__ __align__(256) cnsf::DiagPartial scratch[STATIC_PARTIALS + 1];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
cnsf::DiagPartial* g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on `dev` (which must be current).
int static_scratch(int dev, cnsf::DiagPartial** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(CNSF_E_DEVICE, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = static_cast<cnsf::DiagPartial*>(p);
  }
  *out = g_scratch_dev[dev];
  return CNSF_OK;
}
}  // namespace

extern "C" {

int cnsf_step_diagnostics_static(cnsf_lattice* L, int64_t n, cnsf_diag* d) {
  if (!L || !d) return fail(CNSF_E_INVALID, "NULL argument");
  if (n < 1) return fail(CNSF_E_INVALID, "n = %lld < 1", (long long)n);
  if (L->lc.grid > STATIC_PARTIALS)
    return fail(CNSF_E_SIZE,
                "persistent grid of %d blocks: the static workspace holds the partial sums of at most %d blocks",
                L->lc.grid, STATIC_PARTIALS);
  (void)hipSetDevice(L->device);
  DiagPartial* sp = nullptr;
  if (int r = static_scratch(L->device, &sp)) return r;
  // the update that reduces the level at entry runs on at most STATIC_PARTIALS
  // blocks (a persistent grid when the lattice has more tiles); the populations
  // it writes do not depend on the launch shape
  Launch lc = L->lc;
  uint32_t nb = update_blocks(L->g, lc);
  if (nb > (uint32_t)STATIC_PARTIALS) {
    lc.grid = STATIC_PARTIALS;
    nb = STATIC_PARTIALS;
  }
  const int64_t step0 = L->step;
  hipError_t e = launch_update_diag(L->p.storage, L->pop, L->g, L->ph, L->cd, L->parity, lc, L->phd, sp, nullptr,
                                    L->stream);
  if (e != hipSuccess) return hip_fail(e, "fused diagnostic update");
  L->parity ^= 1;
  ++L->step;
  e = launch_diag_final(sp, (int)nb, sp + STATIC_PARTIALS, L->stream);
  if (e != hipSuccess) return hip_fail(e, "diagnostic reduction");
  if (int r = cnsf_step(L, n - 1)) return r;
  DiagPartial r{};
  e = hipMemcpyAsync(&r, sp + STATIC_PARTIALS, sizeof r, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "step_diagnostics_static");
  fill_diag(L, r, false, step0, d);
  return CNSF_OK;
}

int cnsf_spectrum_shells(const cnsf_lattice* L, int32_t* nshells) {
  if (!L || !nshells) return fail(CNSF_E_INVALID, "NULL argument");
  if (L->g.nx != L->g.ny || L->g.nx != L->g.nz || L->g.bc_x != CNSF_BC_PERIODIC)
    return fail(CNSF_E_INVALID, "the shell spectrum needs a cubic periodic lattice");
  *nshells = (int32_t)spectrum_shells(L->g.nx);
  return CNSF_OK;
}

int cnsf_spectrum(cnsf_lattice* L, double* E, int32_t nshells, int32_t where) {
  if (!L || !E) return fail(CNSF_E_INVALID, "NULL argument");
  int32_t need = 0;
  if (int r = cnsf_spectrum_shells(L, &need)) return r;
  if (nshells < need) return fail(CNSF_E_SIZE, "spectrum needs %d shells, got %d", need, nshells);
  if (where != CNSF_HOST && where != CNSF_DEVICE) return fail(CNSF_E_INVALID, "where must be HOST or DEVICE");
  (void)hipSetDevice(L->device);
  hipError_t e = hipSuccess;
  if (!L->fields) {
    e = hipMalloc(&L->fields, (size_t)8 * L->g.ncells * sizeof(double));
    if (e != hipSuccess) {
      L->fields = nullptr;
      return fail(CNSF_E_NOMEM, "spectral workspace: %s", hipGetErrorString(e));
    }
  }
  const size_t npart = (size_t)L->g.nz * (size_t)need;
  if (!L->spec) {
    e = hipMalloc(&L->spec, (npart + (size_t)need) * sizeof(double));
    if (e != hipSuccess) {
      L->spec = nullptr;
      return fail(CNSF_E_NOMEM, "spectrum partials: %s", hipGetErrorString(e));
    }
  }
  double* dE = where == CNSF_DEVICE ? E : L->spec + npart;
  const uint32_t nout = where == CNSF_DEVICE ? (uint32_t)nshells : (uint32_t)need;
  e = launch_velocity(L->p.storage, L->pop, L->g, L->cd, L->parity, L->fields, L->stream);
  if (e == hipSuccess) e = launch_spectrum(L->g, L->fields, L->spec, dE, nout, L->stream);
  if (e == hipSuccess && where == CNSF_HOST) {
    e = hipMemcpyAsync(E, dE, (size_t)need * sizeof(double), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    for (int32_t k = need; k < nshells; ++k) E[k] = 0.0;
  }
  if (e != hipSuccess) return hip_fail(e, "spectrum");
  return CNSF_OK;
}

int cnsf_get_launch(const cnsf_lattice* L, int32_t* block, int32_t* tile, int32_t* grid, int32_t* xcd_remap) {
  if (!L) return fail(CNSF_E_INVALID, "lattice is NULL");
  if (block) *block = L->lc.block;
  if (tile) *tile = L->lc.tile;
  if (grid) *grid = L->lc.grid;
  if (xcd_remap) *xcd_remap = L->lc.remap;
  return CNSF_OK;
}

int cnsf_get_info(const cnsf_lattice* L, int64_t* step, int32_t* parity, size_t* ckpt) {
  if (!L) return fail(CNSF_E_INVALID, "lattice is NULL");
  if (step) *step = L->step;
  if (parity) *parity = L->parity;
  if (ckpt) *ckpt = L->bytes;
  return CNSF_OK;
}

int cnsf_export_populations(cnsf_lattice* L, void* host, size_t bytes, int64_t* step, int32_t* parity) {
  if (!L || !host) return fail(CNSF_E_INVALID, "NULL argument");
  if (bytes != L->bytes) return fail(CNSF_E_SIZE, "checkpoint buffer %zu != %zu bytes", bytes, L->bytes);
  (void)hipSetDevice(L->device);
  hipError_t e = hipMemcpyAsync(host, L->pop, bytes, hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "export");
  if (step) *step = L->step;
  if (parity) *parity = L->parity;
  return CNSF_OK;
}

int cnsf_import_populations(cnsf_lattice* L, const void* host, size_t bytes, int64_t step, int32_t parity) {
  if (!L || !host) return fail(CNSF_E_INVALID, "NULL argument");
  if (bytes != L->bytes) return fail(CNSF_E_SIZE, "checkpoint of %zu bytes != %zu", bytes, L->bytes);
  if (parity != 0 && parity != 1) return fail(CNSF_E_INVALID, "parity %d", parity);
  (void)hipSetDevice(L->device);
  hipError_t e = hipMemcpyAsync(L->pop, host, bytes, hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "import");
  L->step = step;
  L->parity = parity;
  return CNSF_OK;
}

int cnsf_hbm_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src) return fail(CNSF_E_INVALID, "NULL argument");
  if (bytes % 16) return fail(CNSF_E_INVALID, "bytes %zu not a multiple of 16", bytes);
  hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "copy");
  return CNSF_OK;
}

const char* cnsf_last_error(void) { return cnsf::last_error(); }

const char* cnsf_status_string(int s) {
  switch (s) {
    case CNSF_OK: return "ok";
    case CNSF_E_INVALID: return "invalid argument";
    case CNSF_E_NOMEM: return "out of memory or buffer too small";
    case CNSF_E_DEVICE: return "HIP error";
    case CNSF_E_STATE: return "invalid state (rho <= 0, p <= 0 or non-finite)";
    case CNSF_E_SIZE: return "size mismatch";
    default: return "unknown status";
  }
}

}  // extern "C"
