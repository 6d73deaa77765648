// What fixes the update's memory traffic besides its kernels: the population
// layout (region stride) and the default launch shape of each storage type.
#include <hip/hip_runtime.h>

#include "../../include/cnsf.h"
#include "api_common.h"
#include "cnsf_impl.h"
#include "launch.h"

namespace cnsf {

Launch default_launch(int storage) {
  // Measured on the 512^3 update with the grouped slot layout: one block per
  // tile throughout; 256-cell tiles dealt to the XCDs in contiguous spans for
  // FP32 and BF16, 512-cell tiles in hardware order for FP16.
  Launch lc;
  lc.block = 256;
  lc.tile = 256;
  lc.grid = 0;
  lc.remap = 1;
  if (storage == CNSF_STORAGE_FP16) {
    lc.tile = 512;
    lc.remap = 0;
  }
  return lc;
}

// Elements between consecutive component regions: 7 slots of the cell count
// rounded up to whole slot groups.
uint64_t component_stride(uint64_t ncells, int storage) {
  (void)storage;
  return (uint64_t)NV * ((ncells + SLOT_GROUP - 1) / SLOT_GROUP * SLOT_GROUP);
}

}  // namespace cnsf
