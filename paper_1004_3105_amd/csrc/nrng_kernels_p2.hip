// nrng_kernels_p2.hip -- the method P2 (Section 4) mask and generate kernel instances (templates in
// nrng_kernels.hpp), compiled in a translation unit of their own.
#include "nrng_kernels.hpp"

namespace nrng {

const void *polar_gen_ptr_p2(int mode, int dtype, int vi) { return polar_gen_vm<VM_P2>(mode, dtype, vi); }
const void *polar_mask_ptr_p2(int mode, int vi) { return polar_mask_vm<VM_P2>(mode, vi); }

}  // namespace nrng
