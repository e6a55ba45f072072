// MFMA helpers shared by the block kernels (block_kernels.hip, block_sym_*.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace phmg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 step and the accumulator's element -> tile-row map.  Both
// instructions give lane l the column l % 16; float64 stores rows
// l/16 + 4e in element e, float32 rows 4 (l/16) + e.
template <typename Acc>
struct Mfma;
template <>
struct Mfma<double> {
    typedef d4 acc_t;
    __device__ static inline d4 step(double a, double b, d4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int e) { return lane / 16 + 4 * e; }
};
template <>
struct Mfma<float> {
    typedef f4 acc_t;
    __device__ static inline f4 step(float a, float b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int e) { return 4 * (lane / 16) + e; }
};

}  // namespace phmg
