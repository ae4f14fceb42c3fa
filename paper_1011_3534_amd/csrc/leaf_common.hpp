// Device helpers of the leaf-product kernels.
#pragma once

#include "spamm_internal.hpp"

namespace spamm {
namespace leafk {

#define GLOBAL __attribute__((address_space(1)))
#define LDSP __attribute__((address_space(3)))

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

enum Kind { kF64 = 0, kF32 = 1, kBF16 = 2, kBF16X3 = 3, kF16 = 4, kF16X3 = 5 };

constexpr bool is16(int k) { return k >= kBF16; }
constexpr bool isx3(int k) { return k == kBF16X3 || k == kF16X3; }
constexpr bool isf16(int k) { return k == kF16 || k == kF16X3; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Buffer resource over `bytes` bytes from `base` (uniform).  A load whose
// offset lies outside [0, bytes) returns zero without a memory access, so a
// resource with bytes = 0 turns a whole stage load into a no-op.
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ inline int find_product(const ProdDesc* desc, int nprod, int64_t t) {
    int lo = 0, hi = nprod - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Schedule position p of an nb x nb tile grid -> tile (I, J), walking G-row
// panels top to bottom and, inside a panel, G-column blocks left to right
// (row-major inside a block; edge panels and blocks are narrower).  A bijection
// on [0, nb^2): tiles processed together form 2-D neighbourhoods that share
// both A row panels and B column panels in L2.
template <int G = 8>
__device__ inline void block_order(int64_t p, int nb, int& I, int& J) {
    const int64_t panel = p / ((int64_t)G * nb);
    const int64_t rem = p - panel * G * nb;
    const int h = nb - (int)panel * G < G ? nb - (int)panel * G : G;
    const int64_t bj = rem / ((int64_t)h * G);
    const int64_t rem2 = rem - bj * h * G;
    const int w = nb - (int)bj * G < G ? nb - (int)bj * G : G;
    I = (int)(panel * G + rem2 / w);
    J = (int)(bj * G + rem2 % w);
}

}  // namespace leafk
}  // namespace spamm
