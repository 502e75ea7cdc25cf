// Interpolation FMM far field (FP32): placeholder until the tree code lands.
#include "pmx_internal.hpp"

namespace pmx {
struct FMM {};
void fmm_build(pmx_operator*, hipStream_t) { throw Error(PMX_ERR_INVALID, "FMM far field is not available yet"); }
void fmm_destroy(FMM* f) { delete f; }
void fmm_far(pmx_operator*, int, hipStream_t) { throw Error(PMX_ERR_INVALID, "FMM far field is not available yet"); }
void fmm_stats(const FMM*, pmx_operator_stats*) {}
uint64_t fmm_bytes(const FMM*) { return 0; }
}  // namespace pmx
