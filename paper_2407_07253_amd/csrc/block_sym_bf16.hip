// Symmetric-layout block patch solve, __hip_bfloat16 factors (see block_sym.h).
#include "block_sym.h"

namespace phmg {

void launch_block_sym_bf16(hipStream_t s, const Level& L, const double* X, const double* gw) {
    blocksym::launch<__hip_bfloat16, float>(s, L, X, gw);
}

}  // namespace phmg
