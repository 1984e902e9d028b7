// nrng_kernels_b3.hip -- the method B3 (Section 3) kernel instances (templates in
// nrng_kernels.hpp), compiled in a translation unit of their own.
#include "nrng_kernels.hpp"

namespace nrng {

const void *bm_ptr_b3(int batched, int dtype, int vi) { return bm_family_ptr<BM_B3>(batched, dtype, vi); }
const void *bm_words_ptr_b3(int dtype) { return bm_family_words_ptr<BM_B3>(dtype); }

}  // namespace nrng
