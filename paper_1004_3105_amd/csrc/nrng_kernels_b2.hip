// nrng_kernels_b2.hip -- the method B2 (Section 3) kernel instances (templates in
// nrng_kernels.hpp), compiled in a translation unit of their own.
#include "nrng_kernels.hpp"

namespace nrng {

const void *bm_ptr_b2(int batched, int dtype, int vi) { return bm_family_ptr<BM_B2>(batched, dtype, vi); }
const void *bm_words_ptr_b2(int dtype) { return bm_family_words_ptr<BM_B2>(dtype); }

}  // namespace nrng
