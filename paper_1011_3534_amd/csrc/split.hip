// Split 16-bit copies of FP32 tiles for the 16-bit leaf precisions.
//
// A 16-bit leaf product multiplies x = hi + lo with hi and lo in FP16 or
// BF16 (three MFMA products hi*hi + hi*lo + lo*hi for the "x3" variants).
// Every kept product reads whole operand tiles, and one tile is read by many
// products, so the split is made once per tile here, in the tile-major layout
// of the FP32 tiles (hi tiles first, then lo tiles), and the leaf kernel
// copies the halves straight into LDS.
//
// FP16: tile values are first scaled by an exact power of two (f16_shift of
// the tile's exponent) so the largest lies in [2^14, 2^15), away from FP16
// overflow and underflow; the leaf kernel undoes the scales of both operands
// on each product's FP32 partial sum.  BF16 has the FP32 exponent range and
// needs no scaling.  Both halves are rounded to nearest even.
#include "spamm_internal.hpp"

namespace spamm {
namespace {

#define GLOBAL __attribute__((address_space(1)))

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t pack2(uint16_t a, uint16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

// One thread per 8 consecutive elements of the split storage (tile-major,
// row-major inside a tile); the FP32 source is read through the handle's
// tile layout g (packed tiles, or the caller's array for a view).
template <int B, int KIND>
__global__ void __launch_bounds__(256) k_split(const float* __restrict__ tiles, TileGeo g, int64_t nb,
                                               const int8_t* __restrict__ texp, int64_t nunits,
                                               uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                               const int* __restrict__ active) {
    if (active && *active == 0) return;
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= nunits) return;
    const int64_t t = (u * 8) / (B * B);
    const int e = (int)((u * 8) % (B * B));
    const GLOBAL f32x4* src = (const GLOBAL f32x4*)(tiles + g.tile(t / nb, t % nb) + (int64_t)(e / B) * g.ld + e % B);
    const f32x4 x0 = src[0], x1 = src[1];
    int sh = 0;
    if constexpr (KIND == kSplitF16) sh = f16_shift(texp[t]);
    float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    uint16_t h[8], l[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) split16<KIND>(KIND == kSplitF16 ? ldexpf(x[j], sh) : x[j], h[j], l[j]);
    u32x4 vh, vl;
    vh.x = pack2(h[0], h[1]);
    vh.y = pack2(h[2], h[3]);
    vh.z = pack2(h[4], h[5]);
    vh.w = pack2(h[6], h[7]);
    vl.x = pack2(l[0], l[1]);
    vl.y = pack2(l[2], l[3]);
    vl.z = pack2(l[4], l[5]);
    vl.w = pack2(l[6], l[7]);
    ((GLOBAL u32x4*)hi)[u] = vh;
    ((GLOBAL u32x4*)lo)[u] = vl;
}

template <int B>
hipError_t split_b(const spamm_matrix* M, int kind, const int* active, hipStream_t s) {
    const int64_t elems = M->nb * M->nb * (int64_t)B * B;
    const int64_t nunits = elems / 8;
    const unsigned blocks = (unsigned)((nunits + 255) / 256);
    uint16_t* hi = M->split;
    uint16_t* lo = M->split + elems;
    if (kind == kSplitF16)
        hipLaunchKernelGGL((k_split<B, kSplitF16>), dim3(blocks), dim3(256), 0, s, (const float*)M->tiles,
                           tile_geo(M), M->nb, M->texp, nunits, hi, lo, active);
    else
        hipLaunchKernelGGL((k_split<B, kSplitBF16>), dim3(blocks), dim3(256), 0, s, (const float*)M->tiles,
                           tile_geo(M), M->nb, M->texp, nunits, hi, lo, active);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_split(const spamm_matrix* M, int kind, const int* active, hipStream_t s) {
    if (M->dt != SPAMM_F32 || !M->split) return hipErrorInvalidValue;
    switch (M->b) {
        case 32: return split_b<32>(M, kind, active, s);
        case 64: return split_b<64>(M, kind, active, s);
        case 128: return split_b<128>(M, kind, active, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace spamm
