// nrng_kernels_p.hip -- the Algorithm P (Section 2) mask and generate kernel instances (templates in
// nrng_kernels.hpp), compiled in a translation unit of their own.
#include "nrng_kernels.hpp"

namespace nrng {

const void *polar_gen_ptr_p(int mode, int dtype, int vi) { return polar_gen_vm<VM_P>(mode, dtype, vi); }
const void *polar_mask_ptr_p(int mode, int vi) { return polar_mask_vm<VM_P>(mode, vi); }

}  // namespace nrng
