// Symmetric-layout block patch solve, double factors (see block_sym.h).
#include "block_sym.h"

namespace phmg {

void launch_block_sym_f64(hipStream_t s, const Level& L, const double* X, const double* gw) {
    blocksym::launch<double, double>(s, L, X, gw);
}

}  // namespace phmg
