// Batched ensembles: many independent periodic lattices advanced by one
// launch per step.
//
// A descriptor table in device memory holds each member's geometry, constants
// and population offset.  Each member's cells are cut into tiles of `tile`
// cells, numbered member after member (prefix sums of the tile counts); a
// second table gives the member of every tile, so a block finds its member
// with one load instead of a search over the prefix sums.  With grid = 0 every
// tile gets its own block; with grid > 0 a fixed grid strides over the tiles
// (persistent within a step).  Steps can be captured once into a HIP graph
// and replayed.  Mode 2 launches the single-lattice update per member, the
// sequential baseline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cnsf.h"
#include "api_common.h"
#include "cnsf_impl.h"
#include "launch.h"

namespace cnsf {

struct Member {
  Geom g;
  Phys ph;
  Codec cd;
  uint64_t pop_offset;  // elements from the batch base
  uint32_t tile0;       // first tile of this member
  uint32_t ntiles;
};

template <int ST, bool SC, int PAR>
__global__ void __launch_bounds__(256) k_batch_update(typename Store<ST>::T* __restrict__ base,
                                                      const Member* __restrict__ members,
                                                      const uint16_t* __restrict__ tile_member,
                                                      uint32_t total_tiles, uint32_t tile) {
  constexpr int parity = PAR;
  for (uint32_t t = blockIdx.x; t < total_tiles; t += gridDim.x) {
    const Member& M = members[tile_member[t]];   // uniform per block
    const Geom g = M.g;
    typename Store<ST>::T* pop = base + M.pop_offset;
    const uint32_t first = (t - M.tile0) * tile;
    for (uint32_t j = threadIdx.x; j < tile; j += blockDim.x) {
      const uint32_t c = first + j;
      if (c >= g.ncells) break;
      const Nbr n = neighbours(c, g);
      uint32_t off[NV];
      stream_offsets<ST, 0>(g, n, parity, off);
      float gv[NC][NV];
      gather<ST, 0, SC, float>(pop, g, M.cd, n, parity, off, gv);
      update_cell(gv, M.cd, M.ph);
      scatter<ST, 0, SC>(pop, g, M.cd, M.ph, WallCell{}, n, parity, off, gv);
    }
  }
}

static hipError_t launch_batch(int storage, bool scaled, void* base, const Member* members,
                               const uint16_t* tile_member, uint32_t total_tiles, uint32_t tile, int block, int grid,
                               int parity, hipStream_t s) {
  const uint32_t nb = grid > 0 ? (uint32_t)grid : total_tiles;
#define CNSF_CASE(ST, SC, T)                                                                            \
  if (storage == ST && scaled == SC) {                                                                  \
    if (parity)                                                                                         \
      hipLaunchKernelGGL((k_batch_update<ST, SC, 1>), dim3(nb), dim3(block), 0, s, (T*)base, members,    \
                         tile_member, total_tiles, tile);                                               \
    else                                                                                                \
      hipLaunchKernelGGL((k_batch_update<ST, SC, 0>), dim3(nb), dim3(block), 0, s, (T*)base, members,    \
                         tile_member, total_tiles, tile);                                               \
    return hipGetLastError();                                                                           \
  }
  CNSF_CASE(0, false, float)
  CNSF_CASE(1, false, uint16_t)
  CNSF_CASE(2, false, uint16_t)
  CNSF_CASE(1, true, uint16_t)
  CNSF_CASE(2, true, uint16_t)
#undef CNSF_CASE
  return hipErrorInvalidValue;
}

}  // namespace cnsf

using namespace cnsf;

struct cnsf_batch {
  std::vector<cnsf_params> p;
  std::vector<Member> m;   // host copy
  std::vector<PhysD> phd;
  Member* dm = nullptr;    // device table
  uint16_t* dtile = nullptr;       // member of every tile (device)
  uint32_t dtile_cap = 0;
  int storage = 0;
  void* base = nullptr;
  bool owned = false;
  size_t bytes = 0;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t gstream = nullptr;  // capture stream of the graph
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  int device = 0;
  int parity = 0;
  int64_t step = 0;
  int block = 256;
  uint32_t tile = 256;
  int grid = 0;
  int graph_steps = 20;
  uint32_t total_tiles = 0;
  int* dflag = nullptr;
  bool scaled = false;   // some member stores with a non-unit scale
  bool interleaved = false;  // component-major population layout
};

// Population layout of a batch.  Component-major when every region fits the
// 32-bit offsets of the buffer resources: component k of all members is one
// run, member after member, and consecutive runs start S elements apart, so
// a member's 14 regions lie as far apart as a large lattice's.  S is the
// members' total slot count, or more when the caller's buffer is larger than
// required (up to the 32-bit limit): wider spacing is what lets MI355X run an
// ensemble at the rate of one large lattice.  Otherwise member-major: each
// member's own population array after the previous one.
struct BatchLayout {
  bool interleaved = false;
  uint64_t S = 0;                 // elements between component runs (interleaved)
  std::vector<uint64_t> offset;   // first element of each member's component 0
  size_t bytes = 0;               // bytes the layout occupies
};

static int batch_layout(const cnsf_params* members, int32_t n, size_t avail, BatchLayout& L) {
  const size_t eb = elem_bytes(members[0].storage);
  const uint64_t align = 256 / eb;              // member runs start on 256-byte boundaries
  const uint64_t limit = ((1ull << 32) - 512) / eb / align * align;   // largest S of a 32-bit region
  uint64_t S = 0;
  for (int j = 0; j < n; ++j) {
    const uint64_t nc = (uint64_t)members[j].nx * members[j].ny * members[j].nz;
    S += (component_stride(nc, members[j].storage) + align - 1) / align * align;
  }
  L.offset.assign(n, 0);
  if (S <= limit) {
    L.interleaved = true;
    uint64_t off = 0;
    for (int j = 0; j < n; ++j) {
      const uint64_t nc = (uint64_t)members[j].nx * members[j].ny * members[j].nz;
      L.offset[j] = off;
      off += (component_stride(nc, members[j].storage) + align - 1) / align * align;
    }
    const uint64_t wide = avail / ((uint64_t)NC * eb) / align * align;
    L.S = std::max(S, std::min(wide, limit));
    L.bytes = (size_t)NC * L.S * eb;
    return CNSF_OK;
  }
  uint64_t off = 0;
  for (int j = 0; j < n; ++j) {
    size_t nb = 0;
    if (int e = cnsf_required_bytes(&members[j], &nb)) return e;
    L.offset[j] = off;
    off += (nb + 255) / 256 * 256 / eb;
  }
  L.bytes = (size_t)off * eb;
  return CNSF_OK;
}

static void batch_drop_graph(cnsf_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
}

static int batch_retile(cnsf_batch* b) {
  uint32_t t0 = 0;
  std::vector<uint16_t> owner;
  for (size_t j = 0; j < b->m.size(); ++j) {
    Member& M = b->m[j];
    M.tile0 = t0;
    M.ntiles = (M.g.ncells + b->tile - 1) / b->tile;
    t0 += M.ntiles;
    owner.insert(owner.end(), M.ntiles, (uint16_t)j);
  }
  b->total_tiles = t0;
  hipError_t e = hipSuccess;
  if (b->dtile_cap < t0) {
    if (b->dtile) (void)hipFree(b->dtile);
    b->dtile = nullptr;
    b->dtile_cap = 0;
    e = hipMalloc(&b->dtile, sizeof(uint16_t) * t0);
    if (e != hipSuccess) return fail(CNSF_E_NOMEM, "tile table: %s", hipGetErrorString(e));
    b->dtile_cap = t0;
  }
  e = hipMemcpy(b->dtile, owner.data(), sizeof(uint16_t) * t0, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->dm, b->m.data(), sizeof(Member) * b->m.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  batch_drop_graph(b);
  return CNSF_OK;
}

static hipError_t batch_launch_steps(cnsf_batch* b, int64_t n, hipStream_t s, int& parity) {
  for (int64_t i = 0; i < n; ++i) {
    hipError_t e = launch_batch(b->storage, b->scaled, b->base, b->dm, b->dtile, b->total_tiles, b->tile,
                                b->block, b->grid, parity, s);
    if (e != hipSuccess) return e;
    parity ^= 1;
  }
  return hipSuccess;
}

extern "C" {

int cnsf_batch_required_bytes(const cnsf_params* members, int32_t n, size_t* bytes) {
  if (!members || n < 1 || !bytes) return fail(CNSF_E_INVALID, "batch needs n >= 1 members");
  if (n > 65536) return fail(CNSF_E_INVALID, "%d members: a batch holds at most 65536", n);
  for (int j = 0; j < n; ++j) {
    size_t nb = 0;
    if (int e = cnsf_required_bytes(&members[j], &nb)) return e;
    if (members[j].storage != members[0].storage) return fail(CNSF_E_INVALID, "members differ in storage");
    if (members[j].bc_x != CNSF_BC_PERIODIC) return fail(CNSF_E_INVALID, "batch members must be periodic");
  }
  BatchLayout L;
  if (int e = batch_layout(members, n, 0, L)) return e;
  *bytes = L.bytes;
  return CNSF_OK;
}

int cnsf_batch_create(const cnsf_params* members, int32_t n, void* dev_buf, size_t bytes, void* stream,
                      cnsf_batch** out) {
  if (!out) return fail(CNSF_E_INVALID, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  if (int e = cnsf_batch_required_bytes(members, n, &need)) return e;
  if (dev_buf && bytes < need) return fail(CNSF_E_NOMEM, "buffer of %zu bytes < required %zu", bytes, need);
  if (dev_buf && ((uintptr_t)dev_buf & 255u)) return fail(CNSF_E_INVALID, "buffer not 256-byte aligned");
  auto* b = new cnsf_batch();
  b->storage = members[0].storage;
  b->stream = (hipStream_t)stream;
  b->bytes = need;
  (void)hipGetDevice(&b->device);
  BatchLayout lay;
  (void)batch_layout(members, n, dev_buf ? bytes : 0, lay);   // validated by cnsf_batch_required_bytes above
  b->bytes = lay.bytes;
  b->interleaved = lay.interleaved;
  for (int j = 0; j < n; ++j) {
    const cnsf_params* p = &members[j];
    b->p.push_back(*p);
    PhysD d = derive_phys_d(p);
    b->phd.push_back(d);
    Member M{};
    M.g = derive_geom(p, d);
    if (lay.interleaved) M.g.cstride = lay.S;   // component k of member j at offset[j] + k S
    M.ph = to_float(d);
    M.cd = derive_codec(p, d);
    M.pop_offset = lay.offset[j];
    if (M.cd.scaled) b->scaled = true;
    b->m.push_back(M);
  }
  hipError_t e;
  if (dev_buf) {
    b->base = dev_buf;
  } else {
    e = hipMalloc(&b->base, need);
    if (e != hipSuccess) {
      delete b;
      return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    }
    b->owned = true;
  }
  e = hipMalloc(&b->dm, sizeof(Member) * n);
  if (e == hipSuccess) e = hipMalloc(&b->dflag, sizeof(int));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    cnsf_batch_destroy(b);
    return fail(CNSF_E_NOMEM, "batch buffers: %s", hipGetErrorString(e));
  }
  if (int r = batch_retile(b)) {
    cnsf_batch_destroy(b);
    return r;
  }
  // padding slots are never written by a step; cleared, exports are deterministic
  e = hipMemsetAsync(b->base, 0, b->bytes, b->stream);
  if (e != hipSuccess) {
    cnsf_batch_destroy(b);
    return hip_fail(e, "clearing the population array");
  }
  *out = b;
  return CNSF_OK;
}

int cnsf_batch_destroy(cnsf_batch* b) {
  if (!b) return CNSF_OK;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->gstream) (void)hipStreamSynchronize(b->gstream);
  batch_drop_graph(b);
  if (b->owned && b->base) (void)hipFree(b->base);
  if (b->dm) (void)hipFree(b->dm);
  if (b->dtile) (void)hipFree(b->dtile);
  if (b->dflag) (void)hipFree(b->dflag);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  delete b;
  return CNSF_OK;
}

int cnsf_batch_set_state(cnsf_batch* b, int32_t j, const double* Q, int32_t where) {
  if (!b || !Q) return fail(CNSF_E_INVALID, "NULL argument");
  if (j < 0 || j >= (int)b->m.size()) return fail(CNSF_E_INVALID, "member %d of %zu", j, b->m.size());
  if (where != CNSF_HOST && where != CNSF_DEVICE) return fail(CNSF_E_INVALID, "where = %d", where);
  if (b->parity != 0) return fail(CNSF_E_INVALID, "set_state on a batch at odd parity; set every member before stepping");
  (void)hipSetDevice(b->device);
  const Member& M = b->m[j];
  const size_t qbytes = (size_t)NC * M.g.ncells * sizeof(double);
  const double* dQ = Q;
  double* tmp = nullptr;
  hipError_t e = hipSuccess;
  if (where == CNSF_HOST) {
    e = hipMalloc(&tmp, qbytes);
    if (e != hipSuccess) return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", qbytes, hipGetErrorString(e));
    e = hipMemcpyAsync(tmp, Q, qbytes, hipMemcpyHostToDevice, b->stream);
    dQ = tmp;
  }
  int bad = 0;
  void* pop = (char*)b->base + M.pop_offset * elem_bytes(b->storage);
  if (e == hipSuccess) e = hipMemsetAsync(b->dflag, 0, sizeof(int), b->stream);
  if (e == hipSuccess) e = launch_init(b->storage, pop, dQ, M.g, b->phd[j], M.cd, 0, M.g.ncells, b->dflag, false, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, b->dflag, sizeof(int), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "batch set_state");
  if (bad) return fail(CNSF_E_STATE, "member %d: rho <= 0, p <= 0 or a non-finite value", j);
  return CNSF_OK;
}

int cnsf_batch_set_launch(cnsf_batch* b, int32_t block, int32_t tile, int32_t grid, int32_t graph_steps) {
  if (!b) return fail(CNSF_E_INVALID, "batch is NULL");
  if (block < 64 || block > 256 || block % 64) return fail(CNSF_E_INVALID, "block %d not a multiple of 64 in [64, 256]", block);
  if (tile < block || tile % block) return fail(CNSF_E_INVALID, "tile %d must be a multiple of block %d", tile, block);
  if (grid < 0) return fail(CNSF_E_INVALID, "grid %d", grid);
  if (graph_steps < 2 || graph_steps % 2) return fail(CNSF_E_INVALID, "graph_steps %d must be even >= 2", graph_steps);
  b->block = block;
  b->grid = grid;
  b->graph_steps = graph_steps;
  if ((uint32_t)tile != b->tile) {
    b->tile = tile;
    return batch_retile(b);
  }
  batch_drop_graph(b);
  return CNSF_OK;
}

int cnsf_batch_get_launch(const cnsf_batch* b, int32_t* block, int32_t* tile, int32_t* grid, int32_t* graph_steps) {
  if (!b) return fail(CNSF_E_INVALID, "batch is NULL");
  if (block) *block = b->block;
  if (tile) *tile = (int32_t)b->tile;
  if (grid) *grid = b->grid;
  if (graph_steps) *graph_steps = b->graph_steps;
  return CNSF_OK;
}

int cnsf_batch_step(cnsf_batch* b, int64_t n, int32_t mode) {
  if (!b) return fail(CNSF_E_INVALID, "batch is NULL");
  if (n < 0 || mode < 0 || mode > 2) return fail(CNSF_E_INVALID, "n %lld, mode %d", (long long)n, mode);
  (void)hipSetDevice(b->device);
  hipError_t e = hipSuccess;
  if (mode == 2) {
    for (int64_t s = 0; s < n && e == hipSuccess; ++s) {
      for (size_t j = 0; j < b->m.size() && e == hipSuccess; ++j) {
        const Member& M = b->m[j];
        void* pop = (char*)b->base + M.pop_offset * elem_bytes(b->storage);
        Launch lc;
        lc.block = b->block;
        lc.tile = (int)b->tile;
        lc.grid = 0;
        lc.remap = 1;
        e = launch_update(b->storage, pop, M.g, M.ph, M.cd, b->parity, lc, b->stream);
      }
      b->parity ^= 1;
    }
  } else if (mode == 0) {
    e = batch_launch_steps(b, n, b->stream, b->parity);
  } else {
    int64_t left = n;
    // graphs start at even parity and hold an even number of steps
    if (left > 0 && b->parity) {
      e = batch_launch_steps(b, 1, b->stream, b->parity);
      --left;
    }
    const int64_t reps = left / b->graph_steps;
    if (e == hipSuccess && reps > 0) {
      if (!b->gexec) {
        hipGraph_t graph = nullptr;
        int par = 0;
        e = hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          hipError_t el = batch_launch_steps(b, b->graph_steps, b->gstream, par);
          e = hipStreamEndCapture(b->gstream, &graph);
          if (el != hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (e == hipSuccess) e = hipEventRecord(b->ev_in, b->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->gstream, b->ev_in, 0);
      for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(b->gexec, b->gstream);
      if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->gstream);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_out, 0);
      left -= reps * b->graph_steps;
    }
    if (e == hipSuccess && left > 0) e = batch_launch_steps(b, left, b->stream, b->parity);
  }
  if (e != hipSuccess) return hip_fail(e, "batch step");
  b->step += n;
  return CNSF_OK;
}

int cnsf_batch_get_moments(cnsf_batch* b, int32_t j, double* out, int32_t where) {
  if (!b || !out) return fail(CNSF_E_INVALID, "NULL argument");
  if (j < 0 || j >= (int)b->m.size()) return fail(CNSF_E_INVALID, "member %d of %zu", j, b->m.size());
  (void)hipSetDevice(b->device);
  const Member& M = b->m[j];
  const size_t qbytes = (size_t)NC * M.g.ncells * sizeof(double);
  double* dst = out;
  double* tmp = nullptr;
  hipError_t e = hipSuccess;
  if (where == CNSF_HOST) {
    e = hipMalloc(&tmp, qbytes);
    if (e != hipSuccess) return fail(CNSF_E_NOMEM, "hipMalloc(%zu): %s", qbytes, hipGetErrorString(e));
    dst = tmp;
  }
  const void* pop = (const char*)b->base + M.pop_offset * elem_bytes(b->storage);
  e = launch_moments(b->storage, pop, dst, M.g, M.cd, b->parity, 0, M.g.ncells, b->stream);
  if (e == hipSuccess && tmp) e = hipMemcpyAsync(out, tmp, qbytes, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "batch get_moments");
  return CNSF_OK;
}

// Shape signature of a batch: storage and the sorted member sizes.
static std::string batch_signature(const cnsf_batch* b) {
  std::vector<uint32_t> sizes;
  for (const auto& M : b->m) sizes.push_back(M.g.ncells);
  std::sort(sizes.begin(), sizes.end());
  std::ostringstream os;
  os << "s" << b->storage << "_n" << sizes.size();
  uint64_t h = 1469598103934665603ull;
  for (uint32_t s : sizes) {
    h ^= s;
    h *= 1099511628211ull;
  }
  os << "_" << std::hex << h;
  return os.str();
}

static bool cache_lookup(const char* path, const std::string& key, int& block, int& tile, int& grid) {
  if (!path) return false;
  std::ifstream in(path);
  if (!in) return false;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string s = ss.str();
  const size_t pos = s.find("\"" + key + "\"");
  if (pos == std::string::npos) return false;
  return sscanf(s.c_str() + pos + key.size() + 2, " : {\"block\": %d, \"tile\": %d, \"grid\": %d}", &block, &tile,
                &grid) == 3;
}

static void cache_store(const char* path, const std::string& key, int block, int tile, int grid) {
  if (!path) return;
  std::string body;
  {
    std::ifstream in(path);
    if (in) {
      std::stringstream ss;
      ss << in.rdbuf();
      body = ss.str();
    }
  }
  char entry[256];
  snprintf(entry, sizeof entry, "\"%s\": {\"block\": %d, \"tile\": %d, \"grid\": %d}", key.c_str(), block, tile, grid);
  const size_t close = body.rfind('}');
  if (body.empty() || close == std::string::npos) {
    body = std::string("{\n  ") + entry + "\n}\n";
  } else {
    const bool empty = body.find('"') == std::string::npos;
    body = body.substr(0, close);
    while (!body.empty() && (body.back() == '\n' || body.back() == ' ')) body.pop_back();
    body += (empty ? "\n  " : ",\n  ") + std::string(entry) + "\n}\n";
  }
  std::ofstream out(path);
  out << body;
}

int cnsf_batch_autotune(cnsf_batch* b, const char* cache_path, int32_t steps_per_trial) {
  if (!b) return fail(CNSF_E_INVALID, "batch is NULL");
  if (steps_per_trial < 2) steps_per_trial = 2;
  steps_per_trial += steps_per_trial % 2;
  (void)hipSetDevice(b->device);
  const std::string key = batch_signature(b);
  int bb, tt, gg;
  if (cache_lookup(cache_path, key, bb, tt, gg)) return cnsf_batch_set_launch(b, bb, tt, gg, b->graph_steps);
  // trial steps change the state: keep a copy and restore it afterwards
  void* save = nullptr;
  hipError_t e = hipMalloc(&save, b->bytes);
  if (e != hipSuccess) return fail(CNSF_E_NOMEM, "autotune copy of %zu bytes: %s", b->bytes, hipGetErrorString(e));
  e = hipMemcpyAsync(save, b->base, b->bytes, hipMemcpyDeviceToDevice, b->stream);
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
  struct Cand { int block, tile, grid; };
  std::vector<Cand> cands;
  for (int blk : {64, 128, 256})
    for (int mult : {1, 2, 4})
      for (int grd : {0, ncu * 4, ncu * 8}) cands.push_back({blk, blk * mult, grd});
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  float best = 1e30f;
  Cand bestc{b->block, (int)b->tile, b->grid};
  const int parity0 = b->parity;
  for (const Cand& c : cands) {
    if (e != hipSuccess) break;
    if (int r = cnsf_batch_set_launch(b, c.block, c.tile, c.grid, b->graph_steps)) { e = hipErrorInvalidValue; (void)r; break; }
    int par = parity0;
    e = batch_launch_steps(b, 2, b->stream, par);  // warm up
    if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
    if (e == hipSuccess) e = batch_launch_steps(b, steps_per_trial, b->stream, par);
    if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && ms < best) {
      best = ms;
      bestc = c;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e == hipSuccess) e = hipMemcpyAsync(b->base, save, b->bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(save);
  b->parity = parity0;
  if (e != hipSuccess) return hip_fail(e, "autotune");
  if (int r = cnsf_batch_set_launch(b, bestc.block, bestc.tile, bestc.grid, b->graph_steps)) return r;
  cache_store(cache_path, key, bestc.block, bestc.tile, bestc.grid);
  return CNSF_OK;
}

}  // extern "C"
