// nrng_kernels_b1.hip -- the Algorithm B1 (Section 2) kernel instances (templates in
// nrng_kernels.hpp), compiled in a translation unit of their own.
#include "nrng_kernels.hpp"

namespace nrng {

const void *bm_ptr_b1(int batched, int dtype, int vi) { return bm_family_ptr<BM_B1>(batched, dtype, vi); }
const void *bm_words_ptr_b1(int dtype) { return bm_family_words_ptr<BM_B1>(dtype); }

}  // namespace nrng
