// nrng_kernels_r.hip -- the Algorithm R (Section 5) mask and generate kernel instances (templates in
// nrng_kernels.hpp), compiled in a translation unit of their own.
#include "nrng_kernels.hpp"

namespace nrng {

const void *polar_gen_ptr_r(int mode, int dtype, int vi) { return polar_gen_vm<VM_R>(mode, dtype, vi); }
const void *polar_mask_ptr_r(int mode, int vi) { return polar_mask_vm<VM_R>(mode, vi); }

}  // namespace nrng
