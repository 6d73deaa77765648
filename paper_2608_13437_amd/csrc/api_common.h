// Helpers shared by the lattice and batch halves of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/cnsf.h"
#include "cnsf_impl.h"

namespace cnsf {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const char* last_error();
size_t elem_bytes(int storage);
uint64_t component_stride(uint64_t ncells, int storage);
int validate(const cnsf_params* p);
PhysD derive_phys_d(const cnsf_params* p);
Phys to_float(const PhysD& d);
Geom derive_geom(const cnsf_params* p, const PhysD& ph);
Codec derive_codec(const cnsf_params* p, const PhysD& ph);

}  // namespace cnsf
