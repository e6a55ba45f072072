// Symmetric-layout block patch solve, float factors (see block_sym.h).
#include "block_sym.h"

namespace phmg {

void launch_block_sym_f32(hipStream_t s, const Level& L, const double* X, const double* gw) {
    blocksym::launch<float, float>(s, L, X, gw);
}

}  // namespace phmg
