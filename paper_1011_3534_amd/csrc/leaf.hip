// Dense leaf products of SpAMM (the finest tier of Eq. 4) on gfx950 MFMA.
//
// One 256-thread workgroup owns one C tile (I, J): it lists the kept K of the
// tile in ascending order from the leaf bitmask written by the cull, streams
// A_IK and B_KJ through double-buffered LDS in k-chunks, with the global loads
// of two chunks in flight, and accumulates with 16x16 MFMA blocks; the four
// waves split the tile 2 x 2.  Operand pointers are cast to the global address
// space so the loads are global (not flat) loads: flat loads would also count
// against the LDS wait counter and serialise the MFMA chunk with the prefetch.
// Tiles are handed out XCD by XCD (block x runs on XCD x mod 8), each XCD
// taking a contiguous run of tiles so that neighbouring tiles, which share
// operand panels, meet in the same L2.
//
// The epilogue stages the tile through LDS, stores it coalesced, and computes
// its FP64 squared norm in the same fixed order as the build (per column over
// ascending rows with FMA, then the pairwise column tree), so the result can
// be an operand of the next product with norms identical to a fresh build of
// the stored values.  The SP2 variant also applies the TC2 update
// X <- X^2 or 2X - X^2 and emits FP64 partials of ||X^2 - X||_F^2 and tr(X).
#include "leaf_common.hpp"

namespace spamm {
namespace {

using namespace leafk;

// Geometry of one (leaf size, precision) instance.
template <int B, int P>
struct Geo {
    static constexpr int R = B / 32;                                   // 16x16 blocks per wave per dim
    static constexpr int KC = (P == kF64) ? (B == 128 ? 16 : 32) : 32;  // k-chunk (small: 3 blocks per CU)
    static constexpr int NCH = B / KC;                                 // chunks per task
    // operand element in LDS
    using E = typename std::conditional<P == kF64, double, typename std::conditional<is16(P), uint16_t, float>::type>::type;
    // row strides (elements); 16-bit rows are unpadded and swizzled (sw16).
    // FP32 A rows are 34 words apart: the 16 rows of an MFMA fragment read
    // at one k fall on 16 distinct banks (34 r mod 32 = 2 r), which a 36-word
    // stride would map pairwise (r and r + 8) onto the same bank.
    static constexpr int SA = is16(P) ? KC : KC + 2;
    static constexpr int SB = (P == kF64) ? B + 8 : (is16(P) ? KC : B + 16);
    static constexpr int ROWS_B = is16(P) ? B : KC;                                // B^T rows for 16-bit
    static constexpr int NARR = isx3(P) ? 2 : 1;                                   // hi (+ lo)
    static constexpr int A_ELEMS = B * SA;
    static constexpr int B_ELEMS = ROWS_B * SB;
    static constexpr int BUF_BYTES = NARR * (A_ELEMS + B_ELEMS) * (int)sizeof(E);
    using CT = typename std::conditional<P == kF64, double, float>::type;         // accumulator
    static constexpr int SC = B + (P == kF64 ? 2 : 4);                            // C staging stride
    static constexpr int C_BYTES = B * SC * (int)sizeof(CT);
    static constexpr int SMEM = (2 * BUF_BYTES > C_BYTES) ? 2 * BUF_BYTES : C_BYTES;
    static_assert(!is16(P) || KC == 32, "the 16-bit LDS swizzle assumes 32-wide k-chunks");
};

// 16-bit LDS rows (A rows and B^T rows, 32 k = four 16-byte groups; two
// rows per 128 bytes): group g of row r sits at slot g ^ q(r) with
// q(r) = ((r >> 1) & 3) ^ ((r >> 3) & 1).  Eight consecutive rows at one
// group fill 128 bytes of banks and sixteen fill 256, and so do two (four)
// rows at all four groups, so the MFMA fragment reads (16 rows, one group)
// and both stores (4 rows x 4 groups, or 64 rows x one group) are free of
// bank conflicts whether the LDS serves 16-byte accesses 8 or 16 lanes at a
// time, with no padding.
__device__ inline int sw16(int r, int k) {
    return (((k >> 3) ^ ((r >> 1) & 3) ^ ((r >> 3) & 1)) << 3) | (k & 7);
}

// Kept K of one segment of a tile's mask (four words), with the FP16 scale
// exponents of A_IK and B_KJ.
struct KList {
    int k[256];
    int16_t sa[256];  // FP16: A_IK is scaled by 2^sa, B_KJ by 2^sb
    int16_t sb[256];
};

// Register stage of one k-chunk, FP32/FP64 leaves: float4/double2-sized units
// of A rows and of B rows.
template <int B, int P, typename TA>
struct Stage {
    using G = Geo<B, P>;
    static constexpr int KC = G::KC;
    static constexpr int VA = 16 / (int)sizeof(TA);
    static constexpr int NU = B * KC / VA;                                // units per operand chunk
    static constexpr int UA = (NU + 255) / 256;                           // units per thread
    static constexpr bool PARTIAL = (NU % 256) != 0;
    TA a[UA][VA];
    TA b[UA][VA];
};

// Register stage of one k-chunk, 16-bit leaves (pre-split hi/lo tiles):
// A units are 8 consecutive k of one row (16 bytes); B units are 8
// consecutive k of a column pair, one 32-bit word per k.
template <int B, int P>
struct Stage16 {
    using G = Geo<B, P>;
    static constexpr int KC = G::KC;
    static constexpr int NA = B * KC / 8;
    static constexpr int UA = (NA + 255) / 256;
    static constexpr bool PA = (NA % 256) != 0;
    static constexpr int NB = (B / 2) * (KC / 8);
    static constexpr int UB = (NB + 255) / 256;
    static constexpr bool PB = (NB % 256) != 0;
    u32x4 a[G::NARR][UA];
    uint32_t b[G::NARR][UB][8];
};

// ra: A tile from the chunk's first column (rows lda apart); rb: B tile
// from the chunk's first row (rows ldb apart).
template <int B, int P, typename TA>
__device__ inline void stage_load(Stage<B, P, TA>& st, __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb,
                                  int tid, int lda, int ldb) {
    using S = Stage<B, P, TA>;
    constexpr int KC = S::KC, VA = S::VA;
#pragma unroll
    for (int u = 0; u < S::UA; ++u) {
        const int unit = tid + u * 256;
        if (S::PARTIAL && unit >= S::NU) break;
        const int r = unit / (KC / VA), k = (unit % (KC / VA)) * VA;
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(ra, (r * lda + k) * (int)sizeof(TA), 0, 0);
        const TA* e = reinterpret_cast<const TA*>(&v);
#pragma unroll
        for (int j = 0; j < VA; ++j) st.a[u][j] = e[j];
    }
#pragma unroll
    for (int u = 0; u < S::UA; ++u) {
        const int unit = tid + u * 256;
        if (S::PARTIAL && unit >= S::NU) break;
        const int k = unit / (B / VA), c = (unit % (B / VA)) * VA;
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rb, (k * ldb + c) * (int)sizeof(TA), 0, 0);
        const TA* e = reinterpret_cast<const TA*>(&v);
#pragma unroll
        for (int j = 0; j < VA; ++j) st.b[u][j] = e[j];
    }
}

template <int B, int P, typename TA>
__device__ inline void stage_store(const Stage<B, P, TA>& st, char* buf, int tid) {
    using G = Geo<B, P>;
    using S = Stage<B, P, TA>;
    using E = typename G::E;
    constexpr int KC = G::KC, VA = S::VA;
    E* As = reinterpret_cast<E*>(buf);
    E* Bs = As + G::A_ELEMS;
#pragma unroll
    for (int u = 0; u < S::UA; ++u) {
        const int unit = tid + u * 256;
        if (S::PARTIAL && unit >= S::NU) break;
        const int r = unit / (KC / VA), k = (unit % (KC / VA)) * VA;
#pragma unroll
        for (int j = 0; j < VA; ++j) As[r * G::SA + k + j] = (E)st.a[u][j];
    }
#pragma unroll
    for (int u = 0; u < S::UA; ++u) {
        const int unit = tid + u * 256;
        if (S::PARTIAL && unit >= S::NU) break;
        const int k = unit / (B / VA), c = (unit % (B / VA)) * VA;
#pragma unroll
        for (int j = 0; j < VA; ++j) Bs[k * G::SB + c + j] = (E)st.b[u][j];
    }
}

// ra[h] / rb[h]: hi (h = 0) and lo (h = 1) tiles as in stage_load.
template <int B, int P>
__device__ inline void stage16_load(Stage16<B, P>& st, const __amdgpu_buffer_rsrc_t* ra,
                                    const __amdgpu_buffer_rsrc_t* rb, int tid) {
    using S = Stage16<B, P>;
    constexpr int KC = S::KC;
#pragma unroll
    for (int h = 0; h < Geo<B, P>::NARR; ++h) {
#pragma unroll
        for (int u = 0; u < S::UA; ++u) {
            const int unit = tid + u * 256;
            if (S::PA && unit >= S::NA) break;
            const int r = unit / (KC / 8), k = (unit % (KC / 8)) * 8;
            st.a[h][u] = __builtin_amdgcn_raw_buffer_load_b128(ra[h], (r * B + k) * 2, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < S::UB; ++u) {
            const int unit = tid + u * 256;
            if (S::PB && unit >= S::NB) break;
            const int cp = unit % (B / 2), k = (unit / (B / 2)) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                st.b[h][u][j] = __builtin_amdgcn_raw_buffer_load_b32(rb[h], (k * (B / 2) + cp) * 4, j * (B / 2) * 4, 0);
        }
    }
}

// A rows go to LDS as loaded; each B unit is transposed into two LDS rows of
// B^T (columns 2cp and 2cp+1, 8 consecutive k each).
template <int B, int P>
__device__ inline void stage16_store(const Stage16<B, P>& st, char* buf, int tid) {
    using G = Geo<B, P>;
    using S = Stage16<B, P>;
    constexpr int KC = G::KC;
    uint16_t* As = reinterpret_cast<uint16_t*>(buf);
    uint16_t* Bs = As + G::NARR * G::A_ELEMS;
#pragma unroll
    for (int h = 0; h < G::NARR; ++h) {
#pragma unroll
        for (int u = 0; u < S::UA; ++u) {
            const int unit = tid + u * 256;
            if (S::PA && unit >= S::NA) break;
            const int r = unit / (KC / 8), k = (unit % (KC / 8)) * 8;
            *reinterpret_cast<u32x4*>(As + h * G::A_ELEMS + r * G::SA + sw16(r, k)) = st.a[h][u];
        }
#pragma unroll
        for (int u = 0; u < S::UB; ++u) {
            const int unit = tid + u * 256;
            if (S::PB && unit >= S::NB) break;
            const int cp = unit % (B / 2), k = (unit / (B / 2)) * 8;
            const uint32_t* w = st.b[h][u];
            u32x4 ev, od;
            ev.x = (w[0] & 0xFFFFu) | (w[1] << 16);
            ev.y = (w[2] & 0xFFFFu) | (w[3] << 16);
            ev.z = (w[4] & 0xFFFFu) | (w[5] << 16);
            ev.w = (w[6] & 0xFFFFu) | (w[7] << 16);
            od.x = (w[0] >> 16) | (w[1] & 0xFFFF0000u);
            od.y = (w[2] >> 16) | (w[3] & 0xFFFF0000u);
            od.z = (w[4] >> 16) | (w[5] & 0xFFFF0000u);
            od.w = (w[6] >> 16) | (w[7] & 0xFFFF0000u);
            // columns 2cp and 2cp+1 share (row >> 2), hence the swizzle
            uint16_t* dst = Bs + h * G::B_ELEMS + (2 * cp) * G::SB + sw16(2 * cp, k);
            *reinterpret_cast<u32x4*>(dst) = ev;
            *reinterpret_cast<u32x4*>(dst + G::SB) = od;
        }
    }
}

// LDS slots (16 bytes) of a stage.  A rows hold 4 slots (32 k); slot s of
// row r sits at s ^ dqa(r), so the 16 rows of an A fragment read spread over
// all banks.  B rows hold 8 slots (64 columns); slot s of row k sits at
// s ^ dfb(k), so the 8 rows of one 32-lane half of a transposing read (rows
// k..k+3 and k+8..k+11) hit disjoint banks.
__device__ inline int dqa(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }
__device__ inline int dfb(int k) { return (((k >> 1) & 1) | (((k >> 3) & 1) << 1)) << 1; }

// Register stage of one k-chunk, 16-bit leaves split on the fly from FP32
// tiles (operands without split tiles): A units are 8 consecutive k of one
// row.  B units are 8 consecutive columns of one k-row at leaf 64 (two
// 16-byte loads; B stays row-major in LDS in the layout of the split-operand
// stages, and the MFMA fragments come from the transposing LDS read), and 8
// consecutive k of one column at leaf 32 and 128 (8 loads, coalesced over c).
template <int B, int P>
struct Stage16c {
    using G = Geo<B, P>;
    static constexpr int KC = G::KC;
    static constexpr int NU = B * KC / 8;
    static constexpr int U = (NU + 255) / 256;
    static constexpr bool PARTIAL = (NU % 256) != 0;
    float a[U][8];
    float b[U][8];
};

template <int B, int P>
__device__ inline void stage16c_load(Stage16c<B, P>& st, __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb,
                                     int tid, int lda, int ldb) {
    using S = Stage16c<B, P>;
    constexpr int KC = S::KC;
#pragma unroll
    for (int u = 0; u < S::U; ++u) {
        const int unit = tid + u * 256;
        if (S::PARTIAL && unit >= S::NU) break;
        const int r = unit / (KC / 8), k = (unit % (KC / 8)) * 8;
        // one lane offset per unit; the constant parts go in the scalar offset
        const int vo = (r * lda + k) * 4;
        const f32x4 v0 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, vo, 0, 0));
        const f32x4 v1 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, vo, 16, 0));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            st.a[u][j] = v0[j];
            st.a[u][4 + j] = v1[j];
        }
    }
    if constexpr (B == 64) {
        // leaf 64: B units are 8 consecutive columns of one k-row (two 16-byte
        // loads), kept row-major in LDS (the MFMA reads transpose them)
        const int k = tid >> 3, c = (tid & 7) * 8;
        const int vo = (k * ldb + c) * 4;
        const f32x4 v0 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, vo, 0, 0));
        const f32x4 v1 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, vo, 16, 0));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            st.b[0][j] = v0[j];
            st.b[0][4 + j] = v1[j];
        }
    } else {
#pragma unroll
        for (int u = 0; u < S::U; ++u) {
            const int unit = tid + u * 256;
            if (S::PARTIAL && unit >= S::NU) break;
            const int c = unit % B, k = (unit / B) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                st.b[u][j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, (k * ldb + c) * 4, j * ldb * 4, 0));
        }
    }
}

// Split (after the FP16 tile scales sa, sb) into the hi (+ lo) LDS arrays.
template <int B, int P>
__device__ inline void stage16c_store(const Stage16c<B, P>& st, char* buf, int tid, int sa, int sb) {
    using G = Geo<B, P>;
    using S = Stage16c<B, P>;
    constexpr int KC = G::KC;
    constexpr int KIND = isf16(P) ? kSplitF16 : kSplitBF16;
    uint16_t* As = reinterpret_cast<uint16_t*>(buf);
    uint16_t* Bs = As + G::NARR * G::A_ELEMS;
    auto put = [&](const float* x, int s, uint16_t* dh, uint16_t* dl) {
        // pairs: one packed conversion for hi and one for lo
        uint32_t h[4], l[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            spamm_f2 v = {x[2 * j], x[2 * j + 1]};
            if constexpr (isf16(P)) v = spamm_f2{ldexpf(v.x, s), ldexpf(v.y, s)};
            split16x2<KIND>(v, h[j], l[j]);
        }
        *reinterpret_cast<u32x4*>(dh) = u32x4{h[0], h[1], h[2], h[3]};
        if constexpr (isx3(P)) *reinterpret_cast<u32x4*>(dl) = u32x4{l[0], l[1], l[2], l[3]};
    };
#pragma unroll
    for (int u = 0; u < S::U; ++u) {
        const int unit = tid + u * 256;
        if (S::PARTIAL && unit >= S::NU) break;
        const int r = unit / (KC / 8), k = (unit % (KC / 8)) * 8;
        const int ka = sw16(r, k);
        put(st.a[u], sa, As + r * G::SA + ka, As + G::A_ELEMS + r * G::SA + ka);
    }
    if constexpr (B == 64) {
        // row k of B, columns c..c+7 at slot (c / 8) ^ dfb(k) of the row (the
        // layout the transposing fragment reads of stage_mma expect)
        const int k = tid >> 3, cg = tid & 7;
        const int ob = (k * 8 + (cg ^ dfb(k))) * 8;
        put(st.b[0], sb, Bs + ob, Bs + G::B_ELEMS + ob);
    } else {
#pragma unroll
        for (int u = 0; u < S::U; ++u) {
            const int unit = tid + u * 256;
            if (S::PARTIAL && unit >= S::NU) break;
            const int c = unit % B, k = (unit / B) * 8;
            const int kb = sw16(c, k);
            put(st.b[u], sb, Bs + c * G::SB + kb, Bs + G::B_ELEMS + c * G::SB + kb);
        }
    }
}

// MFMA accumulation of one k-chunk held in LDS.
template <int B, int P, typename Acc>
__device__ inline void chunk_mma(const char* buf, Acc (&acc)[Geo<B, P>::R][Geo<B, P>::R], int lane, int wr, int wc) {
    using G = Geo<B, P>;
    using E = typename G::E;
    constexpr int R = G::R, KC = G::KC;
    const E* As = reinterpret_cast<const E*>(buf);
    const E* Bs = As + G::NARR * G::A_ELEMS;
    const int row0 = wr * (B / 2) + (lane & 15);
    const int col0 = wc * (B / 2) + (lane & 15);
    const int g = lane >> 4;
    if constexpr (is16(P)) {
#pragma unroll
        for (int t = 0; t < KC / 32; ++t) {
            const int k = 32 * t + 8 * g;
            using V8 = typename std::conditional<P == kBF16 || P == kBF16X3, bf16x8, f16x8>::type;
            V8 ah[R], bh[R], al[R], bl[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int ra = row0 + 16 * i, rb = col0 + 16 * i;
                const int oa = ra * G::SA + sw16(ra, k), ob = rb * G::SB + sw16(rb, k);
                ah[i] = *reinterpret_cast<const V8*>(As + oa);
                bh[i] = *reinterpret_cast<const V8*>(Bs + ob);
                if constexpr (isx3(P)) {
                    al[i] = *reinterpret_cast<const V8*>(As + G::A_ELEMS + oa);
                    bl[i] = *reinterpret_cast<const V8*>(Bs + G::B_ELEMS + ob);
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if constexpr (P == kBF16 || P == kBF16X3) {
                        if constexpr (isx3(P)) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        }
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                    } else {
                        if constexpr (isx3(P)) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        }
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                    }
                }
        }
    } else {
#pragma unroll
        for (int t = 0; t < KC / 4; ++t) {
            const int k = 4 * t + g;
            E a[R], b[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                a[i] = As[(row0 + 16 * i) * G::SA + k];
                b[i] = Bs[k * G::SB + col0 + 16 * i];
            }
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if constexpr (P == kF64)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                }
        }
    }
}

// Split 16-bit operands at leaf 64 go from memory straight into LDS
// (buffer loads with an LDS destination: no registers, no arithmetic) through
// a ring of NS stages, each holding one 32-wide k-chunk of A_IK (64 rows x 32
// k) and of B_KJ (32 k-rows x 64 columns) for hi and lo.  Each wave issues the
// PW 1 KiB loads of one array of a stage; the ring keeps NS - 1 stages in
// flight.  Two stages and four blocks per CU measured best (more stages cost
// blocks per CU, which hide more of each tile's latency chain).  B stays row-major in LDS: its MFMA fragments (8 consecutive k of
// one column per lane) come from the transposing 16-bit LDS read, which hands
// lane j of each 16-lane group element j % 4 of what lane 4e + j / 4 read, so
// lane i of a group reads row i / 4 of a 4-row slab at columns 4 (i % 4).
template <int B, int P, bool PS>
struct Dma {
    static constexpr bool ON = PS && B == 64 && is16(P);
    static constexpr int NARR = isx3(P) ? 2 : 1;
    static constexpr int ARR = 4096;                 // bytes of one array's chunk
    static constexpr int STAGE = 2 * NARR * ARR;     // A arrays, then B arrays
    static constexpr int NS = 2;
    static constexpr int PW = STAGE / 1024 / 4;      // 1 KiB loads per wave per stage
    static constexpr int SMEM = NS * STAGE;
};

template <int B, int P, bool PS>
constexpr int leaf_smem() {
    return Dma<B, P, PS>::ON ? (Dma<B, P, PS>::SMEM > Geo<B, P>::C_BYTES ? Dma<B, P, PS>::SMEM : Geo<B, P>::C_BYTES)
                             : Geo<B, P>::SMEM;
}

// Byte offset, inside a tile chunk, of the 16 bytes that land at position p
// of the array's LDS chunk (p = 64 * load + lane).
template <bool IS_A>
__device__ inline uint32_t dma_src(int p) {
    if constexpr (IS_A) {
        const int r = p >> 2, sl = (p & 3) ^ dqa(r);
        return (uint32_t)((r * 64 + sl * 8) * 2);
    } else {
        const int k = p >> 3, sl = (p & 7) ^ dfb(k);
        return (uint32_t)((k * 64 + sl * 8) * 2);
    }
}

// MFMA accumulation of one stage (the same products in the same order as
// chunk_mma, so the results are the same bits).
template <int P, typename Acc>
__device__ inline void stage_mma(const char* __restrict__ st, Acc (&acc)[2][2], int lane, int wr, int wc) {
    constexpr int NARR = isx3(P) ? 2 : 1, ARR = 4096;
    using V8 = typename std::conditional<P == kBF16 || P == kBF16X3, bf16x8, f16x8>::type;
    typedef short s16x4 __attribute__((ext_vector_type(4)));
    const int g = lane >> 4, i16 = lane & 15;
    V8 ah[2], bh[2], al[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int r = wr * 32 + 16 * i + i16;
        const int off = (r * 4 + (g ^ dqa(r))) * 16;
        ah[i] = *reinterpret_cast<const V8*>(st + off);
        if constexpr (NARR == 2) al[i] = *reinterpret_cast<const V8*>(st + ARR + off);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int n = wc * 32 + 16 * j + 4 * (i16 & 3);
        s16x4 h2[2], l2[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 8 * g + 4 * h + (i16 >> 2);
            const int off = (k * 8 + ((n >> 3) ^ dfb(k))) * 16 + (n & 7) * 2;
            h2[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LDSP s16x4*)(st + NARR * ARR + off));
            if constexpr (NARR == 2)
                l2[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LDSP s16x4*)(st + (NARR + 1) * ARR + off));
        }
        bh[j] = __builtin_bit_cast(V8, __builtin_shufflevector(h2[0], h2[1], 0, 1, 2, 3, 4, 5, 6, 7));
        if constexpr (NARR == 2)
            bl[j] = __builtin_bit_cast(V8, __builtin_shufflevector(l2[0], l2[1], 0, 1, 2, 3, 4, 5, 6, 7));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if constexpr (P == kBF16 || P == kBF16X3) {
                if constexpr (NARR == 2) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            } else {
                if constexpr (NARR == 2) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        }
}

// s_waitcnt with vmcnt = v (lgkmcnt = 0, expcnt untouched): the wave's own
// LDS reads are done and at most v of its memory loads are outstanding.
template <int V>
__device__ inline void wait_vm_lgkm0() {
    static_assert(V >= 0 && V < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((V & 15) | ((V >> 4) << 14) | (0x7 << 4));
}

// Undo the FP16 scales of the product ending at step t (when t is its last
// chunk) and add its fresh sum to the tile sum: the finish of leaf_tile.
template <int P, int NCH, typename Acc>
__device__ __forceinline__ void finish_product(const KList* __restrict__ kl, int t, Acc (&part)[2][2],
                                               Acc (&acc)[2][2]) {
    if (t % NCH != NCH - 1) return;
    if constexpr (isf16(P)) {
        const int un = __builtin_amdgcn_readfirstlane(-((int)kl->sa[t / NCH] + (int)kl->sb[t / NCH]));
        if (un >= -126 && un <= 127) {
            const float f = ldexpf(1.0f, un);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[i][j][q] = __builtin_fmaf(part[i][j][q], f, acc[i][j][q]);
        } else {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[i][j][q] += ldexpf(part[i][j][q], un);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] += part[i][j];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) part[i][j] = Acc{0, 0, 0, 0};
}

// One step of the direct-to-LDS pipeline: issue this wave's loads of step
// t + NS - 1 into stage `nxt` (past the last step: empty resources, which
// load nothing), then, for t >= 0, the MFMA of stage `cur` and the finish of
// a product.  The restrict qualifiers tell the compiler that the stage being
// read, the stage being loaded and the K list are disjoint, so it adds no
// wait of its own for the loads in flight; the caller's wait and barrier
// order each stage's loads before its reads.
template <int P, int NCH, int PW, typename Acc>
__device__ __forceinline__ void dma_step(const char* __restrict__ cur, char* __restrict__ nxt,
                                         const KList* __restrict__ kl, int t, int T, int NS,
                                         const uint16_t* __restrict__ base16, bool isA, int64_t I, int64_t J, int64_t nb,
                                         const uint32_t (&voff)[PW], Acc (&part)[2][2], Acc (&acc)[2][2],
                                         int lane, int wr, int wc) {
    const int ti = t + NS - 1;
    const bool live = ti < T;
    const int tt = live ? ti : T - 1;
    const int k = __builtin_amdgcn_readfirstlane(kl->k[tt / NCH]);
    const int ch = tt % NCH;
    const int64_t tile = isA ? I * nb + k : (int64_t)k * nb + J;
    const uint32_t coff = isA ? (uint32_t)ch * 64u : (uint32_t)ch * 4096u;
    const __amdgpu_buffer_rsrc_t r = rsrc((const char*)(base16 + tile * 4096) + coff, live ? 8192u - coff : 0u);
#pragma unroll
    for (int q = 0; q < PW; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (LDSP void*)(nxt + q * 1024), 16, voff[q], 0, 0, 0);
    if (t >= 0) {
        stage_mma<P, Acc>(cur, part, lane, wr, wc);
        finish_product<P, NCH, Acc>(kl, t, part, acc);
    }
}

// The thread index as a value the compiler cannot see through.  A persistent
// loop over tiles then derives the per-thread offsets of each tile afresh
// instead of holding them in registers across the loop, which made the leaf
// 64 list kernel spill at four blocks per CU.
__device__ inline int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// One C tile from its kept K to its stored values and norm.  t is a global
// schedule position (blocked = true: panel/block order inside each product)
// or a global tile index (blocked = false: row-major); tid is threadIdx.x.
template <int B, int P, typename TA, typename TC, bool SP2, bool PRESPLIT>
__device__ __forceinline__ void leaf_tile(const ProdDesc* __restrict__ desc, int nprod, int64_t t, char* smem,
                                          KList* kl, double (*red)[4], const int* __restrict__ branch,
                                          bool blocked, int tid) {
    using G = Geo<B, P>;
    using CT = typename G::CT;
    using Acc = typename std::conditional<P == kF64, f64x4, f32x4>::type;
    constexpr int R = G::R, KC = G::KC, NCH = G::NCH;
    const int m = nprod > 1 ? find_product(desc, nprod, t) : 0;
    const ProdDesc& d = desc[m];
    const int nb = d.nb;
    int I, J;
    if (blocked) {
        block_order<8>(t - d.tile_base, nb, I, J);
    } else {
        I = (int)((t - d.tile_base) / nb);
        J = (int)((t - d.tile_base) % nb);
    }
    const int64_t local = (int64_t)I * nb + J;
    const int lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
    const int64_t lo16 = (int64_t)nb * nb * B * B;  // hi tiles -> lo tiles
    constexpr int64_t TS = (int64_t)B * B;
    // Operand tiles, in bytes: A tile (I, k) at a_row + k*a_sk and B tile
    // (k, J) at b_col + k*b_si (both strides below 2^32, checked on the
    // host), rows lda (ldb) elements apart, ext_a (ext_b) bytes from a tile's
    // first element to one past its last.  Computed once here, so the loop
    // adds one scalar product per operand and step.
    constexpr int ESZ = is16(P) ? 4 : (int)sizeof(TA);
    const int lda = (int)d.ga.ld, ldb = (int)d.gb.ld;
    const char* const a_row = (const char*)d.A + d.ga.si * I * ESZ;
    const char* const b_col = (const char*)d.B + d.gb.sk * J * ESZ;
    const uint32_t a_sk = (uint32_t)(d.ga.sk * ESZ), b_si = (uint32_t)(d.gb.si * ESZ);
    const uint32_t ext_a = (uint32_t)(((int64_t)(B - 1) * lda + B) * ESZ);
    const uint32_t ext_b = (uint32_t)(((int64_t)(B - 1) * ldb + B) * ESZ);
    const uint32_t kc_b = (uint32_t)(G::KC * ldb * ESZ);  // bytes between B chunks

    Acc acc[R][R], part[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            acc[i][j] = Acc{0, 0, 0, 0};
            part[i][j] = Acc{0, 0, 0, 0};
        }

    // The kept K of this tile, a segment of four mask words (256 K) at a
    // time, become a list in LDS (with the FP16 scales of each product), so
    // that the pipelined loop issues no global load besides operand chunks.
    const uint64_t* mrow = d.mask + local * d.W;
    bool counted = false;
    for (int w0 = 0; w0 < d.W; w0 += 4) {
        uint64_t wd[4];
        int pre[4], nk = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            wd[j] = (w0 + j < d.W) ? mrow[w0 + j] : 0ull;
            pre[j] = nk;
            nk += __popcll(wd[j]);
        }
        // the FP16 scale exponents of every candidate K of this wave's word,
        // loaded with the mask words (one round trip instead of two)
        const int kc = (w0 + w) * 64 + lane;
        int ea = 0, eb = 0;
        if constexpr (isf16(P)) {
            if (kc < nb) {
                ea = d.eA[(int64_t)I * nb + kc];
                eb = d.eB[(int64_t)kc * nb + J];
            }
        }
        if (nk == 0) continue;
        if (!counted) {
            counted = true;
            if (tid == 0 && d.nonempty) atomicAdd(d.nonempty, 1ull);
        }
        {
            // wave w lists the K of word w0 + w in ascending order
            const uint64_t mine = w == 0 ? wd[0] : w == 1 ? wd[1] : w == 2 ? wd[2] : wd[3];
            const int base = w == 0 ? pre[0] : w == 1 ? pre[1] : w == 2 ? pre[2] : pre[3];
            if ((mine >> lane) & 1ull) {
                // set bits of the word below this lane (mbcnt: no 64-bit lane
                // mask held in registers across the tile)
                const int pos = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mine >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mine, 0u));
                kl->k[pos] = kc;
                if constexpr (isf16(P)) {
                    kl->sa[pos] = (int16_t)f16_shift(ea);
                    kl->sb[pos] = (int16_t)f16_shift(eb);
                }
            }
        }
        __syncthreads();

        // step t = (list entry t / NCH, k-chunk t % NCH); T is uniform, and
        // the loop control stays in scalar registers
        const int T = __builtin_amdgcn_readfirstlane(nk * NCH);
        if constexpr (Dma<B, P, PRESPLIT>::ON) {
            using D = Dma<B, P, PRESPLIT>;
            constexpr int NS = D::NS, PW = D::PW, NARR = D::NARR;
            // this wave's array (x3: A hi, A lo, B hi, B lo; one half: two
            // waves per operand) and its first load in it
            // (the wave index is uniform: readfirstlane keeps everything derived
            // from it, the load resources and LDS bases, in scalar registers)
            const int wu = __builtin_amdgcn_readfirstlane(w);
            const int arr = NARR == 2 ? wu : (wu >> 1);
            const bool isA = arr < NARR;
            const int half = isA ? arr : arr - NARR;
            const int first = NARR == 2 ? 0 : (wu & 1) * PW;
            uint32_t voff[PW];
#pragma unroll
            for (int q = 0; q < PW; ++q) {
                const int p = 64 * (first + q) + lane;
                voff[q] = isA ? dma_src<true>(p) : dma_src<false>(p);
            }
            const uint16_t* base16 = (isA ? d.A16 : d.B16) + half * lo16;
            const int lds0 = arr * D::ARR + first * 1024;
            for (int t = -(NS - 1); t < T; ++t) {
                if (t >= 0) {
                    // this wave's loads of stage t have landed; after the
                    // barrier every wave's have, and every wave is done with
                    // step t - 1, whose stage the next loads overwrite
                    wait_vm_lgkm0<PW * (NS - 2)>();
                    __builtin_amdgcn_sched_barrier(0);
                    __builtin_amdgcn_s_barrier();
                    __builtin_amdgcn_sched_barrier(0);
                    asm volatile("" ::: "memory");
                }
                const int cs = ((t % NS) + NS) % NS, ns = (t + NS - 1) % NS;
                dma_step<P, NCH, PW>(smem + cs * D::STAGE, smem + ns * D::STAGE + lds0, kl, t, T, NS, base16, isA,
                                     I, J, nb, voff, part, acc, lane, wr, wc);
            }
        } else {
        // MFMA on the chunk in LDS buffer bf.  No branches: the scheduler can
        // interleave it with the split and store of the next chunk.
        auto mma = [&](int bf) {
            if constexpr (is16(P) && !PRESPLIT && B == 64)
                stage_mma<P, Acc>(smem + bf * G::BUF_BYTES, part, lane, wr, wc);
            else if constexpr (P != kF64)
                chunk_mma<B, P, Acc>(smem + bf * G::BUF_BYTES, part, lane, wr, wc);
            else
                chunk_mma<B, P, Acc>(smem + bf * G::BUF_BYTES, acc, lane, wr, wc);
        };
        // After the last chunk of a leaf product (step t; `odd`: t is odd, which
        // decides it at compile time for one or two chunks per product) its
        // fresh accumulator is added to the tile sum (two-level summation: the
        // rounding error does not grow with the number of kept products).
        auto fin = [&](int t, bool odd) {
            if constexpr (P != kF64) {
                const bool last = NCH == 1 || (NCH == 2 ? odd : t % NCH == NCH - 1);
                if (last) {
                    const int un = isf16(P) ? __builtin_amdgcn_readfirstlane(
                                                  -((int)kl->sa[t / NCH] + (int)kl->sb[t / NCH]))
                                            : 0;
                    if constexpr (isf16(P)) {
                        // undo the product's power-of-two scales: one FMA by 2^un
                        // when 2^un is a normal float (the same value as ldexpf)
                        if (un >= -126 && un <= 127) {
                            const float f = ldexpf(1.0f, un);
#pragma unroll
                            for (int i = 0; i < R; ++i)
#pragma unroll
                                for (int j = 0; j < R; ++j)
#pragma unroll
                                    for (int q = 0; q < 4; ++q)
                                        acc[i][j][q] = __builtin_fmaf(part[i][j][q], f, acc[i][j][q]);
                        } else {
#pragma unroll
                            for (int i = 0; i < R; ++i)
#pragma unroll
                                for (int j = 0; j < R; ++j)
#pragma unroll
                                    for (int q = 0; q < 4; ++q) acc[i][j][q] += ldexpf(part[i][j][q], un);
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < R; ++i)
#pragma unroll
                            for (int j = 0; j < R; ++j) acc[i][j] += part[i][j];
                    }
#pragma unroll
                    for (int i = 0; i < R; ++i)
#pragma unroll
                        for (int j = 0; j < R; ++j) part[i][j] = Acc{0, 0, 0, 0};
                }
            }
        };
        // Two register stages keep two chunks of loads in flight while LDS
        // double-buffers the chunk under MFMA and the next one.
        using St16 = typename std::conditional<PRESPLIT, Stage16<B, P>, Stage16c<B, P>>::type;
        using St = typename std::conditional<is16(P), St16, Stage<B, P, TA>>::type;
        // Loads are issued for every step t < T + 3 (those past the end with
        // empty resources, which load nothing), so that every path through
        // the loop has the same loads in flight and the waits before each LDS
        // store need only cover the older stage.
        auto ld = [&](St& st, int t) {
            const bool live = t < T;
            const int tt = live ? t : T - 1;
            const int k = __builtin_amdgcn_readfirstlane(kl->k[tt / NCH]);
            const int ch = tt % NCH;
            const char* pa = a_row + (uint64_t)(uint32_t)k * a_sk + ch * (KC * ESZ);
            const char* pb = b_col + (uint64_t)(uint32_t)k * b_si + ch * kc_b;
            const uint32_t na = live ? ext_a - ch * (KC * ESZ) : 0u;
            const uint32_t nbb = live ? ext_b - ch * kc_b : 0u;
            if constexpr (is16(P) && !PRESPLIT) {
                stage16c_load<B, P>(st, rsrc(pa, na), rsrc(pb, nbb), tid, lda, ldb);
            } else if constexpr (is16(P)) {
                // split tiles are always packed
                (void)pa;
                (void)pb;
                const int64_t ta = ((int64_t)I * nb + k) * TS, tb = ((int64_t)k * nb + J) * TS;
                const uint32_t na16 = live ? (uint32_t)((TS - ch * KC) * 2) : 0u;
                const uint32_t nb16 = live ? (uint32_t)((TS - ch * KC * B) * 2) : 0u;
                __amdgpu_buffer_rsrc_t ra[2], rb[2];
#pragma unroll
                for (int h = 0; h < G::NARR; ++h) {
                    ra[h] = rsrc(d.A16 + h * lo16 + ta + ch * KC, na16);
                    rb[h] = rsrc(d.B16 + h * lo16 + tb + (int64_t)ch * KC * B, nb16);
                }
                stage16_load<B, P>(st, ra, rb, tid);
            } else {
                stage_load<B, P, TA>(st, rsrc(pa, na), rsrc(pb, nbb), tid, lda, ldb);
            }
        };
        // (step t's FP16 scales apply when splitting on the fly; a store past
        // the last step stores the empty stage, with the last entry's scales)
        auto sto = [&](const St& st, int bf, int t) {
            if constexpr (is16(P) && !PRESPLIT) {
                const int e = min(t / NCH, nk - 1);
                stage16c_store<B, P>(st, smem + bf * G::BUF_BYTES, tid,
                                     isf16(P) ? __builtin_amdgcn_readfirstlane((int)kl->sa[e]) : 0,
                                     isf16(P) ? __builtin_amdgcn_readfirstlane((int)kl->sb[e]) : 0);
            } else if constexpr (is16(P)) {
                stage16_store<B, P>(st, smem + bf * G::BUF_BYTES, tid);
            } else {
                stage_store<B, P, TA>(st, smem + bf * G::BUF_BYTES, tid);
            }
        };
        // Invariant at the top of each half step: LDS buffer `buf` holds step
        // t, one register stage holds (or is receiving) step t + 1 and the
        // other step t + 2.  A stage is refilled right after it is stored, so
        // both stages stay live throughout (their registers are never reused
        // for other values) and every load has two steps to arrive.
        St s0, s1;
        ld(s0, 0);
        sto(s0, 0, 0);
        __syncthreads();
        ld(s0, 1);
        __builtin_amdgcn_sched_barrier(0);  // stage s0 is the older one on every path
        ld(s1, 2);
        __builtin_amdgcn_sched_barrier(0);
        int buf = 0;
        // (scheduling barriers keep each stage's loads ahead of the MFMA work
        // they overlap; no exit follows a refill of s0 before s1 is refilled,
        // so on every path s0's loads are older than s1's)
        // (each half step runs the MFMA of one chunk, the split and store of
        // the next, which no branch separates, and then the product's finish;
        // the store in the first half runs also when it is past the end)
        for (int t = 0;; t += 2) {
            __builtin_amdgcn_sched_barrier(0);
            mma(buf);
            sto(s0, buf ^ 1, t + 1);
            fin(t, false);
            if (t + 1 >= T) break;
            __syncthreads();
            buf ^= 1;
            if (t + 2 >= T) {
                mma(buf);
                fin(t + 1, true);
                break;
            }
            ld(s0, t + 3);
            __builtin_amdgcn_sched_barrier(0);
            mma(buf);
            sto(s1, buf ^ 1, t + 2);
            fin(t + 1, true);
            __syncthreads();
            buf ^= 1;
            ld(s1, t + 4);
            __builtin_amdgcn_sched_barrier(0);
        }
        }
        // Drain the memory counters: no load issued in this segment is still
        // pending, so the wait analysis at the top of the next segment's loop
        // need not assume one (it would otherwise wait for every load in flight).
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // stage buffers and the list are free again
    }

    // A C tile with no kept product is zero (SP2: when its X tile is zero as
    // well).  If the result handle's exponent says the stored tile already
    // holds zeros from an earlier write, only the zero norm (and SP2's zero
    // partials) are stored.  Fresh handles start with exponents 0 ("not known
    // zero"), so every tile is written at least once.  Static schedule only
    // (one tile per block, so the early exit ends the block); the persistent
    // kernel always runs the full epilogue.
    const bool zero_kept =
        __builtin_amdgcn_readfirstlane((int)(!counted && d.eC[local] == -128 && (!SP2 || d.eA[local] == -128))) != 0;
    if (blocked && zero_kept) {
        if (tid == 0) {
            d.SC[local] = 0.0;
            if constexpr (SP2) {
                d.sp2_part[local] = 0.0;
                if (I == J) d.sp2_part[(int64_t)nb * nb + I] = 0.0;
            }
        }
        return;
    }

    // ---------------------------------------------------------------- epilogue
    CT* Cs = reinterpret_cast<CT*>(smem);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // result layout: f32 16x16x4 / 16x16x32 give row 4*(lane/16) + q,
                // f64 16x16x4 gives row 4*q + lane/16 (column lane%16 in both)
                const int r = wr * (B / 2) + 16 * i + (P == kF64 ? 4 * q + (lane >> 4) : 4 * (lane >> 4) + q);
                const int c = wc * (B / 2) + 16 * j + (lane & 15);
                Cs[r * G::SC + c] = (CT)acc[i][j][q];
            }
    __syncthreads();

    GLOBAL TC* Cg = (GLOBAL TC*)d.C + local * TS;
    constexpr int VC = 16 / (int)sizeof(TC);
    // largest |value| in the stored type (exact: max commutes with widening)
    TC mx = (TC)0;
    double idem = 0.0;
    const GLOBAL TC* Xg = SP2 ? (const GLOBAL TC*)d.X + local * TS : nullptr;
    const int br = SP2 ? *branch : 0;
    for (int u = tid; u < B * B / VC; u += 256) {
        const int r = u / (B / VC), c = (u % (B / VC)) * VC;
        TC v[VC];
#pragma unroll
        for (int j = 0; j < VC; ++j) v[j] = (TC)Cs[r * G::SC + c + j];
        if constexpr (SP2) {
#pragma unroll
            for (int j = 0; j < VC; ++j) {
                const TC xv = Xg[r * B + c + j];
                const double dv = (double)v[j] - (double)xv;
                idem = __fma_rn(dv, dv, idem);
                v[j] = br ? (TC)(xv + xv - v[j]) : v[j];
                Cs[r * G::SC + c + j] = (CT)v[j];
            }
        }
#pragma unroll
        for (int j = 0; j < VC; ++j) {
            mx = fmax(mx, fabs(v[j]));
            Cg[r * B + c + j] = v[j];
        }
    }
    // symmetric squaring: tile (J, I) below the diagonal is the transpose of
    // this one (rows of C_JI from the columns of the staged tile; lanes walk
    // the rows so the LDS reads are conflict-free)
    const bool mirror = d.sym_upper && I < J;
    if (SP2 || mirror) __syncthreads();
    if (mirror) {
        GLOBAL TC* Mg = (GLOBAL TC*)d.C + ((int64_t)J * nb + I) * TS;
        for (int u = tid; u < B * B / VC; u += 256) {
            const int r = u % B, c = (u / B) * VC;
            TC v[VC];
#pragma unroll
            for (int j = 0; j < VC; ++j) v[j] = (TC)Cs[(c + j) * G::SC + r];
#pragma unroll
            for (int j = 0; j < VC; ++j) Mg[r * B + c + j] = v[j];
        }
    }

    // block reductions in a fixed order (deterministic)
    for (int dd = 32; dd >= 1; dd >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, dd, 64));
        if constexpr (SP2) idem += __shfl_down(idem, dd, 64);
    }
    if (lane == 0) {
        red[0][w] = (double)mx;
        red[1][w] = idem;
    }
    // canonical squared norm of the stored tile: wave 0, one (or two) columns per lane
    double s_tile = 0.0;  // (tid 0: the tile's norm, which a NaN anywhere in it makes NaN)
    if (w == 0) {
        double s = 0.0;
        if (lane < B) {
            if constexpr (B == 128) {
                double s2 = 0.0;
                for (int r = 0; r < B; ++r) {
                    const double a0 = (double)(TC)Cs[r * G::SC + lane];
                    const double a1 = (double)(TC)Cs[r * G::SC + lane + 64];
                    s = __fma_rn(a0, a0, s);
                    s2 = __fma_rn(a1, a1, s2);
                }
                s = s + s2;  // tree step h = 64
            } else {
                // rows in ascending order, their loads issued 16 at a time
                for (int r0 = 0; r0 < B; r0 += 16) {
                    CT v[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) v[j] = Cs[(r0 + j) * G::SC + lane];
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const double a0 = (double)(TC)v[j];
                        s = __fma_rn(a0, a0, s);
                    }
                }
            }
        }
        constexpr int H0 = (B == 128 ? 64 : B) / 2;
        for (int h = H0; h >= 1; h >>= 1) {
            const double o = __shfl_down(s, h, 64);
            if (lane < h) s = s + o;
        }
        double tr = 0.0;
        if constexpr (SP2) {
            if (I == J) {
                // trace partial: diagonal of the updated tile, pairwise over lanes
                double dv = 0.0;
                if (lane < B) dv = (double)(TC)Cs[lane * G::SC + lane];
                if constexpr (B == 128) dv += (double)(TC)Cs[(lane + 64) * G::SC + lane + 64];
                for (int h = 32; h >= 1; h >>= 1) {
                    const double o = __shfl_down(dv, h, 64);
                    if (lane < h) dv = dv + o;
                }
                tr = dv;
            }
        }
        if (lane == 0) {
            d.SC[local] = s;
            s_tile = s;
            if constexpr (SP2) {
                if (I == J) d.sp2_part[(int64_t)nb * nb + I] = tr;
            }
        }
    } else if (w == 1 && mirror) {
        // canonical squared norm of the mirrored tile: its column c is row c
        // of the staged tile, summed over its rows in ascending order
        double s = 0.0;
        if (lane < B) {
            if constexpr (B == 128) {
                double s2 = 0.0;
                for (int r = 0; r < B; ++r) {
                    const double a0 = (double)(TC)Cs[lane * G::SC + r];
                    const double a1 = (double)(TC)Cs[(lane + 64) * G::SC + r];
                    s = __fma_rn(a0, a0, s);
                    s2 = __fma_rn(a1, a1, s2);
                }
                s = s + s2;
            } else {
                for (int r = 0; r < B; ++r) {
                    const double a0 = (double)(TC)Cs[lane * G::SC + r];
                    s = __fma_rn(a0, a0, s);
                }
            }
        }
        constexpr int H0 = (B == 128 ? 64 : B) / 2;
        for (int h = H0; h >= 1; h >>= 1) {
            const double o = __shfl_down(s, h, 64);
            if (lane < h) s = s + o;
        }
        if (lane == 0) d.SC[(int64_t)J * nb + I] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double m2 = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        int e = -128;
        if (m2 > 0.0) {
            e = ilogb(m2);
            e = e < -127 ? -127 : (e > 127 ? 127 : e);
        }
        // fmax passes over NaN: a tile holding NaN is marked "not known zero"
        // through its norm, so a later product rewrites it
        if (s_tile != s_tile) e = 127;
        d.eC[local] = (int8_t)e;
        if constexpr (SP2) d.sp2_part[local] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        if (mirror) {
            d.eC[(int64_t)J * nb + I] = (int8_t)e;
            if constexpr (SP2) d.sp2_part[(int64_t)J * nb + I] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        }
    }
    __syncthreads();  // red and smem are reused by the next tile of a persistent block
}

// Static 16-bit leaves that split their operands while staging fit in 128
// VGPRs, so four blocks share a CU (one wave per SIMD each).  So do static
// FP32 leaves up to leaf 64 (40000 bytes of LDS at leaf 64).  The other
// variants, and the persistent kernels (whose tile loop needs more registers),
// keep the compiler's register choice.
template <int B, int P, bool PS>
constexpr int leaf_min_waves() {
    return ((is16(P) || P == kF32) && B <= 64 && (!PS || Dma<B, P, PS>::ON)) ? 4 : 1;
}

// Static schedule: one block per tile; block x runs on XCD x mod 8 and takes
// tile (x mod 8) * chunk + x / 8, so each XCD walks a contiguous tile range.
template <int B, int P, typename TA, typename TC, bool SP2, bool PS>
__global__ void __launch_bounds__(256, (leaf_min_waves<B, P, PS>())) k_leaf(const ProdDesc* __restrict__ desc, int nprod, int64_t total,
                                              int64_t chunk, const int* __restrict__ branch,
                                              const int* __restrict__ active) {
    __shared__ __attribute__((aligned(16))) char smem[leaf_smem<B, P, PS>()];
    __shared__ KList kl;
    __shared__ double red[2][4];
    if (active && *active == 0) return;
    const int64_t x = blockIdx.x;
    const int64_t t = (x & 7) * chunk + (x >> 3);
    if (t >= total) return;
    leaf_tile<B, P, TA, TC, SP2, PS>(desc, nprod, t, smem, &kl, red, branch, true, (int)threadIdx.x);
}

// Persistent schedule: resident blocks pull positions from a queue counter
// and process tile order[pos] (largest kept-K count first); every block
// leaves once the queue passes `total`.
template <int B, int P, typename TA, typename TC, bool SP2, bool PS>
__global__ void __launch_bounds__(256) k_leaf_queue(const ProdDesc* __restrict__ desc, int nprod, int64_t total,
                                                    const uint32_t* __restrict__ order,
                                                    unsigned long long* __restrict__ queue,
                                                    const int* __restrict__ branch, const int* __restrict__ active) {
    __shared__ __attribute__((aligned(16))) char smem[leaf_smem<B, P, PS>()];
    __shared__ KList kl;
    __shared__ double red[2][4];
    __shared__ long long s_pos;
    if (active && *active == 0) return;
    while (true) {
        if (threadIdx.x == 0) s_pos = (long long)atomicAdd(queue, 1ull);
        __syncthreads();
        const long long pos = s_pos;
        __syncthreads();
        if (pos >= total) break;
        leaf_tile<B, P, TA, TC, SP2, PS>(desc, nprod, order ? (int64_t)order[pos] : (int64_t)pos, smem, &kl, red,
                                         branch, false, opaque_tid());
    }
}

// Resident blocks take the listed C tiles (global tile indices) in a static
// stride; the list and its count come from a tile-list kernel (SP2 steps,
// the list schedule).  Leaf 64 below FP64 is compiled for four blocks per CU
// (no spills) and launched with that many; FP64 for the two its 71.7 KB of
// LDS allow.
template <int B, int P, bool PS>
constexpr int list_blocks_per_cu() {
    return Dma<B, P, PS>::ON ? 4 : (B == 32 ? 4 : (B == 64 ? (P == kF64 ? 2 : 4) : 1));
}

template <int B, int P, typename TA, typename TC, bool SP2, bool PS>
__global__ void __launch_bounds__(256, (B == 64 ? list_blocks_per_cu<B, P, PS>() : 1))
    k_leaf_list(const ProdDesc* __restrict__ desc, int nprod, const uint32_t* __restrict__ list,
                const unsigned* __restrict__ count, unsigned* __restrict__ queue, const int* __restrict__ branch,
                const int* __restrict__ active) {
    __shared__ __attribute__((aligned(16))) char smem[leaf_smem<B, P, PS>()];
    __shared__ KList kl;
    __shared__ double red[2][4];
    __shared__ unsigned s_next;
    if (active && *active == 0) return;
    const int64_t n = (int64_t)*count;
    if (!queue) {
        for (int64_t i = blockIdx.x; i < n; i += gridDim.x)
            leaf_tile<B, P, TA, TC, SP2, PS>(desc, nprod, (int64_t)list[i], smem, &kl, red, branch, false,
                                             opaque_tid());
        return;
    }
    // dynamic: each block pulls its next list position from the queue while
    // it works on the current one (the grab's latency hides behind the
    // tile), so blocks with cheap tiles take more of them; every block
    // leaves once the queue passes the count
    if (threadIdx.x == 0) s_next = atomicAdd(queue, 1u);
    __syncthreads();
    int64_t i = s_next;
    __syncthreads();
    while (i < n) {
        if (threadIdx.x == 0) s_next = atomicAdd(queue, 1u);
        leaf_tile<B, P, TA, TC, SP2, PS>(desc, nprod, (int64_t)list[i], smem, &kl, red, branch, false, opaque_tid());
        __syncthreads();
        i = s_next;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 2 x 2 super-tiles of 16-bit leaf-64 products of operands with split tiles.
//
// One 256-thread block owns the C tiles (I0 + qi, J0 + qj), qi, qj in {0, 1},
// and walks the union of their kept K in ascending order.  For each K the
// split hi (+ lo) tiles of A_(I0+qi)K and B_K(J0+qj) that a kept product needs
// go from memory straight into LDS (buffer loads with an LDS destination, no
// registers), each once for the two products that share it, and wave
// q = 2 qi + qj runs the MFMA of product (I0 + qi, K, J0 + qj), a whole 64 x 64
// C tile, if that product is kept.  The stage layout is that of the one-tile
// kernel per operand tile, so every 16 x 16 block sees the same MFMA sequence
// (stage_mma), the same scale undo and the same epilogue arithmetic as in
// leaf_tile: the results are the same bits.  Per kept product the operand
// bytes halve when all four products of a K are kept.

// Kept K of one mask segment of a super-tile: bit q of f marks product
// (I0 + (q >> 1), K, J0 + (q & 1)) as kept; sa[i] / sb[j] are the FP16 scale
// exponents of A_(I0+i)K and B_K(J0+j).
struct QList {
    int k[256];
    uint8_t f[256];
    int16_t sa[2][256];
    int16_t sb[2][256];
};

template <int P>
struct QDma {
    static constexpr int NARR = isx3(P) ? 2 : 1;
    static constexpr int PANEL = 4096;                // one operand tile's array of a chunk (bytes)
    static constexpr int STAGE = 2 * NARR * 2 * PANEL;  // (A, B) x (hi, lo) x two tiles
    static constexpr int NS = 2;
    static constexpr int PW = STAGE / 1024 / 4;       // 1 KiB loads per wave per stage
    static constexpr int SC = 68;                     // C staging stride (floats)
    static constexpr int C_BYTES = 4 * 64 * SC * 4;
    static constexpr int SMEM = NS * STAGE > C_BYTES ? NS * STAGE : C_BYTES;
};

// MFMA of one stage for the 64 x 64 tile of wave (qi, qj): panels of A tile qi
// and B tile qj (per 16 x 16 block the products and order of stage_mma).
template <int P, typename Acc>
__device__ inline void qdma_mma(const char* __restrict__ st, Acc (&acc)[4][4], int lane, int qi, int qj) {
    using D = QDma<P>;
    constexpr int NARR = D::NARR, PN = D::PANEL;
    using V8 = typename std::conditional<P == kBF16 || P == kBF16X3, bf16x8, f16x8>::type;
    typedef short s16x4 __attribute__((ext_vector_type(4)));
    const int g = lane >> 4, i16 = lane & 15;
    // panels: A hi (two tiles), [A lo], B hi, [B lo]
    const char* ah_p = st + qi * PN;
    const char* al_p = st + (2 + qi) * PN;
    const char* bh_p = st + (2 * NARR + qj) * PN;
    const char* bl_p = st + (2 * NARR + 2 + qj) * PN;
    V8 bh[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = 16 * j + 4 * (i16 & 3);
        s16x4 h2[2], l2[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 8 * g + 4 * h + (i16 >> 2);
            const int off = (k * 8 + ((n >> 3) ^ dfb(k))) * 16 + (n & 7) * 2;
            h2[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LDSP s16x4*)(bh_p + off));
            if constexpr (NARR == 2) l2[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LDSP s16x4*)(bl_p + off));
        }
        bh[j] = __builtin_bit_cast(V8, __builtin_shufflevector(h2[0], h2[1], 0, 1, 2, 3, 4, 5, 6, 7));
        if constexpr (NARR == 2)
            bl[j] = __builtin_bit_cast(V8, __builtin_shufflevector(l2[0], l2[1], 0, 1, 2, 3, 4, 5, 6, 7));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 16 * i + i16;
        const int off = (r * 4 + (g ^ dqa(r))) * 16;
        const V8 ah = *reinterpret_cast<const V8*>(ah_p + off);
        V8 al;
        if constexpr (NARR == 2) al = *reinterpret_cast<const V8*>(al_p + off);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (P == kBF16 || P == kBF16X3) {
                if constexpr (NARR == 2) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
            } else {
                if constexpr (NARR == 2) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], acc[i][j], 0, 0, 0);
            }
        }
    }
}

// One step of the super-tile pipeline: this wave's loads of step t + 1 into
// stage `nxt` (past the last step, or for operand tiles no kept product of
// that step reads: empty resources, which load nothing), then for t >= 0 the
// MFMA of stage `cur` if the wave's product is kept, and after a product's
// last chunk the undo of its scales.  The restrict qualifiers tell the
// compiler that the stage being read, the stage being loaded and the list
// are disjoint, so it adds no wait of its own for the loads in flight.
template <int P>
__device__ __forceinline__ void qdma_step(const char* __restrict__ cur, char* __restrict__ nxt,
                                          const QList* __restrict__ kl, int t, int T,
                                          const uint16_t* __restrict__ base16, bool isA, int arr, int u0, int nu,
                                          int I0, int J0, bool hasI1, bool hasJ1, int nb, const uint32_t (&voff)[4],
                                          f32x4 (&part)[4][4], f32x4 (&acc)[4][4], int lane, int q, int qi, int qj) {
    using D = QDma<P>;
    constexpr int NCH = 2;
    {
        const int ti = t + 1;
        const bool live = ti < T;
        const int tt = live ? ti : T - 1;
        const int e = tt / NCH, ch = tt % NCH;
        const int k = __builtin_amdgcn_readfirstlane(kl->k[e]);
        const unsigned f = live ? (unsigned)__builtin_amdgcn_readfirstlane((int)kl->f[e]) : 0u;
        const uint32_t coff = isA ? (uint32_t)ch * 64u : (uint32_t)ch * 4096u;
#pragma unroll
        for (int uu = 0; uu < 2; ++uu) {
            if (uu >= nu) break;
            const int u = u0 + uu;
            const bool need = isA ? (f & (u ? 0xCu : 0x3u)) != 0 : (f & (u ? 0xAu : 0x5u)) != 0;
            const int It = isA ? ((u && hasI1) ? I0 + 1 : I0) : k;
            const int Jt = isA ? k : ((u && hasJ1) ? J0 + 1 : J0);
            const int64_t tile = (int64_t)It * nb + Jt;
            const __amdgpu_buffer_rsrc_t r = rsrc((const char*)(base16 + tile * 4096) + coff, need ? 8192u - coff : 0u);
            char* dst = nxt + (arr * 2 + u) * D::PANEL;
#pragma unroll
            for (int l = 0; l < 4; ++l)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (LDSP void*)(dst + l * 1024), 16, voff[l], 0, 0, 0);
        }
    }
    if (t < 0) return;
    const unsigned fl = (unsigned)__builtin_amdgcn_readfirstlane((int)kl->f[t / NCH]);
    if ((fl >> q) & 1u) qdma_mma<P>(cur, part, lane, qi, qj);
    if (t % NCH != NCH - 1) return;
    const int e = t / NCH;
    if constexpr (isf16(P)) {
        const int un = __builtin_amdgcn_readfirstlane(-((int)kl->sa[qi][e] + (int)kl->sb[qj][e]));
        if (un >= -126 && un <= 127) {
            const float fs = ldexpf(1.0f, un);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[i][j][c] = __builtin_fmaf(part[i][j][c], fs, acc[i][j][c]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[i][j][c] += ldexpf(part[i][j][c], un);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += part[i][j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[i][j] = f32x4{0, 0, 0, 0};
}

// One super-tile per block; block x runs on XCD x mod 8 and takes position
// (x mod 8) * chunk + x / 8 of the super-tile grid (panel order inside).
template <int P>
__global__ void __launch_bounds__(256, 2) k_leaf_quad(const ProdDesc* __restrict__ desc, int64_t total, int64_t chunk) {
    using D = QDma<P>;
    constexpr int NCH = 2, NS = D::NS, PW = D::PW, NARR = D::NARR;
    static_assert(NS == 2, "a step issues the loads of the next step");
    __shared__ __attribute__((aligned(16))) char smem[D::SMEM];
    __shared__ QList kl;
    const int64_t x = blockIdx.x;
    const int64_t pos = (x & 7) * chunk + (x >> 3);
    if (pos >= total) return;
    const ProdDesc& d = desc[0];
    const int nb = d.nb, nq = (nb + 1) >> 1;
    int QI, QJ;
    block_order<4>(pos, nq, QI, QJ);
    const int I0 = 2 * QI, J0 = 2 * QJ;
    const bool hasI1 = I0 + 1 < nb, hasJ1 = J0 + 1 < nb;
    const int tid = threadIdx.x, lane = tid & 63;
    const int q = __builtin_amdgcn_readfirstlane(tid >> 6), qi = q >> 1, qj = q & 1;
    const int I = I0 + qi, J = J0 + qj;
    const bool mine = I < nb && J < nb;  // this wave's tile exists

    // this wave's loads: panels of one array (x3: A hi, A lo, B hi, B lo; one
    // half: A hi and B hi, two waves each) for both operand tiles u = 0, 1
    const int arr = NARR == 2 ? q : (q >> 1);
    const bool isA = arr < NARR;
    const int half = isA ? arr : arr - NARR;  // hi or lo
    const int u0 = NARR == 2 ? 0 : (q & 1), nu = NARR == 2 ? 2 : 1;
    const int64_t lo16 = (int64_t)nb * nb * 4096;  // hi tiles -> lo tiles (elements)
    const uint16_t* __restrict__ base16 = (isA ? d.A16 : d.B16) + half * lo16;
    uint32_t voff[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int p = 64 * l + lane;
        voff[l] = isA ? dma_src<true>(p) : dma_src<false>(p);
    }
    static_assert(PW == 4 * (NARR == 2 ? 2 : 1), "one or two panels of four loads per wave");

    f32x4 acc[4][4], part[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f32x4{0, 0, 0, 0};
            part[i][j] = f32x4{0, 0, 0, 0};
        }

    // mask rows of the four tiles (a missing tile reads the first tile's
    // words and drops them: the loads stay unconditional scalar loads)
    const int64_t loc[4] = {(int64_t)I0 * nb + J0, (int64_t)I0 * nb + (hasJ1 ? J0 + 1 : J0),
                            (int64_t)(hasI1 ? I0 + 1 : I0) * nb + J0,
                            (int64_t)(hasI1 ? I0 + 1 : I0) * nb + (hasJ1 ? J0 + 1 : J0)};
    const bool has[4] = {true, hasJ1, hasI1, hasI1 && hasJ1};
    const int W = d.W;
    unsigned cnt = 0;  // bit t: tile t has a kept product
    for (int w0 = 0; w0 < W; w0 += 4) {
        // words w0..w0+3 of every tile; m[t]: word w0 + q of tile t
        uint64_t uw[4], m[4];
        int pre[4], nk = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int wi = w0 + j < W ? w0 + j : W - 1;
            uw[j] = 0ull;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint64_t v = (has[t] && w0 + j < W) ? d.mask[loc[t] * W + wi] : 0ull;
                uw[j] |= v;
                cnt |= v != 0ull ? 1u << t : 0u;
                if (j == 0) m[t] = v;
                else if (j == q) m[t] = v;
            }
            pre[j] = nk;
            nk += __popcll(uw[j]);
        }
        // the FP16 scale exponents of every candidate K of this wave's word,
        // loaded with the mask words
        const int kc = (w0 + q) * 64 + lane;
        int ea0 = 0, ea1 = 0, eb0 = 0, eb1 = 0;
        if constexpr (isf16(P)) {
            if (kc < nb) {
                ea0 = d.eA[(int64_t)I0 * nb + kc];
                eb0 = d.eB[(int64_t)kc * nb + J0];
                if (hasI1) ea1 = d.eA[(int64_t)(I0 + 1) * nb + kc];
                if (hasJ1) eb1 = d.eB[(int64_t)kc * nb + J0 + 1];
            }
        }
        if (nk == 0) continue;
        {
            // wave q lists the K of word w0 + q in ascending order
            const uint64_t uu = q == 0 ? uw[0] : q == 1 ? uw[1] : q == 2 ? uw[2] : uw[3];
            const int base = q == 0 ? pre[0] : q == 1 ? pre[1] : q == 2 ? pre[2] : pre[3];
            if ((uu >> lane) & 1ull) {
                const int p = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(uu >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)uu, 0u));
                unsigned f = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) f |= (unsigned)((m[t] >> lane) & 1ull) << t;
                kl.k[p] = kc;
                kl.f[p] = (uint8_t)f;
                if constexpr (isf16(P)) {
                    kl.sa[0][p] = (int16_t)f16_shift(ea0);
                    kl.sa[1][p] = (int16_t)f16_shift(ea1);
                    kl.sb[0][p] = (int16_t)f16_shift(eb0);
                    kl.sb[1][p] = (int16_t)f16_shift(eb1);
                }
            }
        }
        __syncthreads();

        const int T = __builtin_amdgcn_readfirstlane(nk * NCH);
        // step t = (list entry t / NCH, k-chunk t % NCH).  Each step waits for
        // its own stage, then issues the loads of step t + 1 into the other
        // stage (past the end: empty resources, which load nothing) and runs
        // the MFMA of its product if kept; after a product's last chunk its
        // fresh sum joins the tile sum with the scales undone (a product that
        // is not kept left part at +0, and adding it changes nothing).
        for (int t = -(NS - 1); t < T; ++t) {
            if (t >= 0) {
                wait_vm_lgkm0<PW * (NS - 2)>();
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("" ::: "memory");
            }
            const int cs = ((t % NS) + NS) % NS, ns = (t + NS - 1) % NS;
            qdma_step<P>(smem + cs * D::STAGE, smem + ns * D::STAGE, &kl, t, T, base16, isA, arr, u0, nu, I0, J0,
                         hasI1, hasJ1, nb, voff, part, acc, lane, q, qi, qj);
        }
        // no load of this segment is still in flight, every wave is done with
        // the stages and the list
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    // (per wave, its own tile; the barriers are block-wide and unconditional)
    const bool kept = (cnt >> q) & 1u;
    const int64_t local = (int64_t)I * nb + J;
    const bool zero_kept = mine && !kept && d.eC[local] == -128;
    const bool write = mine && !zero_kept;
    float* Cs = reinterpret_cast<float*>(smem) + q * 64 * D::SC;
    if (write) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    Cs[(16 * i + 4 * (lane >> 4) + c) * D::SC + 16 * j + (lane & 15)] = acc[i][j][c];
    }
    __syncthreads();
    if (write) {
        GLOBAL float* Cg = (GLOBAL float*)d.C + local * 4096;
        for (int v = lane; v < 1024; v += 64) {
            const int r = v >> 4, c = (v & 15) * 4;
            *reinterpret_cast<GLOBAL f32x4*>(Cg + r * 64 + c) = *reinterpret_cast<const f32x4*>(Cs + r * D::SC + c);
        }
        // canonical squared norm (lane = column, rows ascending, then the
        // pairwise column tree) and the largest |value|
        double s = 0.0;
        float mx = 0.0f;
        for (int r0 = 0; r0 < 64; r0 += 16) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = Cs[(r0 + j) * D::SC + lane];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double a0 = (double)v[j];
                s = __fma_rn(a0, a0, s);
                mx = fmaxf(mx, fabsf(v[j]));
            }
        }
        for (int dd = 32; dd >= 1; dd >>= 1) {
            mx = fmaxf(mx, __shfl_xor(mx, dd, 64));
            const double o = __shfl_down(s, dd, 64);
            if (lane < dd) s = s + o;
        }
        if (lane == 0) {
            d.SC[local] = s;
            const double m2 = (double)mx;
            int e = -128;
            if (m2 > 0.0) {
                e = ilogb(m2);
                e = e < -127 ? -127 : (e > 127 ? 127 : e);
            }
            if (s != s) e = 127;
            d.eC[local] = (int8_t)e;
        }
    } else if (mine && lane == 0) {
        d.SC[local] = 0.0;
    }
    if (tid == 0 && cnt && d.nonempty) atomicAdd(d.nonempty, (unsigned long long)__popc(cnt));
}

template <int B, int P, typename TA, typename TC, bool SP2, bool PS = false>
hipError_t go(const ProdDesc* d_desc, const LeafPlan& p, hipStream_t s) {
    if (p.list) {
        // a grid of the resident blocks; the stride loop is correct for any grid
        int64_t grid = (int64_t)num_cus() * list_blocks_per_cu<B, P, PS>();
        if (grid > p.total_tiles) grid = p.total_tiles < 1 ? 1 : p.total_tiles;
        hipLaunchKernelGGL((k_leaf_list<B, P, TA, TC, SP2, PS>), dim3((unsigned)grid), dim3(256), 0, s, d_desc,
                           p.count, p.list, p.list_count, p.list_queue, p.d_branch, p.d_active);
        return hipGetLastError();
    }
    if (p.queue) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_leaf_queue<B, P, TA, TC, SP2, PS>, 256, 0);
        if (e != hipSuccess || per_cu < 1) per_cu = 1;
        int64_t grid = (int64_t)num_cus() * per_cu;
        if (grid > p.total_tiles) grid = p.total_tiles < 1 ? 1 : p.total_tiles;
        hipLaunchKernelGGL((k_leaf_queue<B, P, TA, TC, SP2, PS>), dim3((unsigned)grid), dim3(256), 0, s, d_desc, p.count,
                           p.total_tiles, p.order, p.queue, p.d_branch, p.d_active);
        return hipGetLastError();
    }
    if constexpr (B == 64 && is16(P) && !SP2 && PS) {
        if (p.count == 1) {
            // a single product of split operands: 2 x 2 super-tiles
            int64_t nb = (int64_t)llround(sqrt((double)p.total_tiles));
            while (nb * nb > p.total_tiles) --nb;
            while ((nb + 1) * (nb + 1) <= p.total_tiles) ++nb;
            const int64_t nq = (nb + 1) / 2, quads = nq * nq;
            if (quads == 0) return hipSuccess;
            const int64_t chunk = (quads + 7) / 8;
            hipLaunchKernelGGL((k_leaf_quad<P>), dim3((unsigned)(chunk * 8)), dim3(256), 0, s, d_desc, quads, chunk);
            return hipGetLastError();
        }
    }
    const int64_t chunk = (p.total_tiles + 7) / 8;
    const int64_t grid = chunk * 8;
    hipLaunchKernelGGL((k_leaf<B, P, TA, TC, SP2, PS>), dim3((unsigned)grid), dim3(256), 0, s, d_desc, p.count,
                       p.total_tiles, chunk, p.d_branch, p.d_active);
    return hipGetLastError();
}

// 16-bit leaves: operands with current split tiles, or split on the fly from
// the FP32 tiles (always in SP2, whose operands change every step)
template <int B, int P>
hipError_t go16(const ProdDesc* d_desc, const LeafPlan& p, hipStream_t s) {
    if (p.sp2) return go<B, P, float, float, true, false>(d_desc, p, s);
    if (p.presplit) return go<B, P, float, float, false, true>(d_desc, p, s);
    return go<B, P, float, float, false, false>(d_desc, p, s);
}

template <int B>
hipError_t dispatch_b(const ProdDesc* d_desc, const LeafPlan& p, bool a_f64, hipStream_t s) {
    switch (p.prec) {
        case SPAMM_LEAF_F64:
            if (a_f64) return go<B, kF64, double, double, false>(d_desc, p, s);
            return go<B, kF64, float, double, false>(d_desc, p, s);
        case SPAMM_LEAF_F32:
            return p.sp2 ? go<B, kF32, float, float, true>(d_desc, p, s) : go<B, kF32, float, float, false>(d_desc, p, s);
        case SPAMM_LEAF_BF16: return go16<B, kBF16>(d_desc, p, s);
        case SPAMM_LEAF_BF16X3: return go16<B, kBF16X3>(d_desc, p, s);
        case SPAMM_LEAF_F16: return go16<B, kF16>(d_desc, p, s);
        case SPAMM_LEAF_F16X3: return go16<B, kF16X3>(d_desc, p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// a_f64 is carried in the plan via the descriptor of product 0 (all products of
// one launch share operand types).
hipError_t launch_leaf_typed(const ProdDesc* d_desc, const LeafPlan& p, bool a_f64, hipStream_t s) {
    switch (p.b) {
        case 32: return dispatch_b<32>(d_desc, p, a_f64, s);
        case 64: return dispatch_b<64>(d_desc, p, a_f64, s);
        case 128: return dispatch_b<128>(d_desc, p, a_f64, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace spamm
