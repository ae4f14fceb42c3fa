// Internal declarations of the gfx950 SpAMM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/spamm.h"

namespace spamm {

constexpr int kMaxLevels = SPAMM_MAX_LEVELS;
constexpr int kMaxBatch = 128;
constexpr int kWave = 64;

// Status bit latched on the device by a product, surfaced by the next syncing call.
constexpr unsigned kDevCapacity = 2u;

// Frontier key of an octree node: product index m (7 bits) | I | J | K (19 bits each).
__host__ __device__ inline uint64_t node_key(uint32_t m, uint32_t I, uint32_t J, uint32_t K) {
    return ((uint64_t)m << 57) | ((uint64_t)I << 38) | ((uint64_t)J << 19) | (uint64_t)K;
}
__host__ __device__ inline uint32_t key_m(uint64_t k) { return (uint32_t)(k >> 57); }
__host__ __device__ inline uint32_t key_i(uint64_t k) { return (uint32_t)((k >> 38) & 0x7FFFF); }
__host__ __device__ inline uint32_t key_j(uint64_t k) { return (uint32_t)((k >> 19) & 0x7FFFF); }
__host__ __device__ inline uint32_t key_k(uint64_t k) { return (uint32_t)(k & 0x7FFFF); }
constexpr int64_t kMaxNb = (int64_t)1 << 19;
// Cull threshold that keeps exactly the pairs of non-zero FP32 tiles: a
// non-zero FP32 tile has S >= (2^-149)^2, so S_A S_B >= 2^-596 > 1e-300.
constexpr double kPresentTau = 1e-150;

// FP16 leaves: a tile whose largest |x| has binary exponent e (-128 for an
// all-zero tile) is scaled by 2^f16_shift(e), which puts that largest value in
// [2^14, 2^15); the product of two scaled tiles is scaled back exactly.
constexpr int kF16Bias = 14;
__host__ __device__ inline int f16_shift(int e) { return kF16Bias - (e == -128 ? 0 : e); }

// Split 16-bit copies of FP32 tiles read by the 16-bit leaf precisions.
constexpr int kSplitF16 = 0;   // hi = fp16(x 2^s), lo = fp16(x 2^s - hi), s = f16_shift(tile exponent)
constexpr int kSplitBF16 = 1;  // hi = bf16(x), lo = bf16(x - hi)

// x = hi + lo + (rounding of lo), both halves rounded to nearest even; x is
// the (FP16: already scaled) FP32 value.  split16 (one value) and split16x2
// (two values, packed: element 0 in the low half) give the same bits.
template <int KIND>
__device__ inline void split16(float x, uint16_t& hi, uint16_t& lo) {
    if constexpr (KIND == kSplitF16) {
        const _Float16 h = (_Float16)x;
        hi = __builtin_bit_cast(uint16_t, h);
        lo = __builtin_bit_cast(uint16_t, (_Float16)(x - (float)h));
    } else {
        const __bf16 h = (__bf16)x;
        hi = __builtin_bit_cast(uint16_t, h);
        lo = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)h));
    }
}

typedef float spamm_f2 __attribute__((ext_vector_type(2)));
typedef _Float16 spamm_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 spamm_b2 __attribute__((ext_vector_type(2)));

template <int KIND>
__device__ inline void split16x2(spamm_f2 x, uint32_t& hi, uint32_t& lo) {
    if constexpr (KIND == kSplitF16) {
        const spamm_h2 h = __builtin_convertvector(x, spamm_h2);
        const spamm_f2 r = x - __builtin_convertvector(h, spamm_f2);
        hi = __builtin_bit_cast(uint32_t, h);
        lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, spamm_h2));
    } else {
        const spamm_b2 h = __builtin_convertvector(x, spamm_b2);
        const spamm_f2 r = x - __builtin_convertvector(h, spamm_f2);
        hi = __builtin_bit_cast(uint32_t, h);
        lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, spamm_b2));
    }
}

// Where the elements of a handle's tiles live: element (r, c) of tile (I, K)
// is at I*si + K*sk + r*ld + c.  Packed tiles (the library's own storage)
// are b*b apart in (I, K) row-major order with rows b apart; a view reads
// the caller's row-major array, whose rows are ld apart.
struct TileGeo {
    int64_t si, sk, ld;
    int32_t b, pad_;
    __host__ __device__ int64_t tile(int64_t I, int64_t K) const { return I * si + K * sk; }
    __host__ __device__ int64_t at(int64_t row, int64_t col) const {
        return tile(row / b, col / b) + (row % b) * ld + col % b;
    }
};

// Per-product descriptor read by the cull and leaf kernels.  Operand and
// result pyramids share the same tier shapes (equal n and leaf).
struct ProdDesc {
    const void* A;            // tile-major operand tiles
    const void* B;
    void* C;                  // tile-major result tiles
    const double* SA;         // norm pyramids (tier l at lvl_off[l])
    const double* SB;
    double* SC;
    const int8_t* eA;         // per-tile max exponent (fp16 scaling)
    const int8_t* eB;
    int8_t* eC;
    uint64_t* mask;           // leaf bitmask, W words per C tile
    double* sp2_part;         // SP2: per-tile FP64 partials (idempotency, trace)
    const void* X;            // SP2: the operand tiles X_m (== A == B)
    const uint16_t* A16;      // split 16-bit tiles of A and B: hi tiles, then lo
    const uint16_t* B16;      //   tiles at +nb^2 b^2 elements (16-bit leaves only)
    unsigned long long* nonempty;  // count of C tiles with at least one kept product (null: not counted)
    int64_t lvl_off[kMaxLevels];
    int32_t lvl_m[kMaxLevels];
    int64_t tile_base;        // first global C-tile index of this product
    double tau2;
    int32_t nb, L, W;
    int32_t a_f64, b_f64;     // operand tile element types (1 = FP64)
    int32_t depth_tau;        // 1: a node at depth k below the root is tested against tau / 8^k
    int32_t sym_upper;        // 1: symmetric squaring: only tiles I <= J are formed, C_JI = C_IJ^T
    int32_t pad_;
    TileGeo ga, gb;           // layouts of the A and B tiles (C tiles are packed)
};

// Device-side counters of one product launch sequence.
struct DevCounters {
    unsigned long long front_count[kMaxLevels];  // kept nodes stored per tier (frontier sizes)
    unsigned long long survivors[kMaxBatch][kMaxLevels];
    double culled_bound[kMaxBatch];
    unsigned status;
    unsigned pad_;
};

// Scratch a result handle owns for the product that writes it.
struct ProductScratch {
    uint64_t* mask = nullptr;          // nb*nb*W words
    uint64_t* front[2] = {nullptr, nullptr};
    int64_t front_cap = 0;
    DevCounters* ctr = nullptr;
    ProdDesc* desc = nullptr;          // device copy of the descriptor
    ProdDesc host_desc{};              // last uploaded copy
    bool desc_valid = false;
    double* sp2_part = nullptr;        // SP2 partial sums (nb*nb + nb)
};

}  // namespace spamm

struct spamm_matrix {
    int64_t n = 0;
    int32_t b = 0;
    int64_t nb = 0;
    int32_t L = 0;
    spamm_dtype dt = SPAMM_F32;
    size_t elem = 4;
    void* tiles = nullptr;       // packed tiles, or the borrowed array of a view
    bool view = false;           // tiles borrow the caller's row-major array (not owned)
    int64_t ld = 0;              // a view's row stride (elements)
    double* norms = nullptr;
    bool tiers_valid = false;    // tiers above the leaves match the leaf norms (formed on demand)
    int8_t* texp = nullptr;
    uint16_t* split = nullptr;   // split 16-bit tiles (hi, then lo), made on demand
    int split_kind = -1;         // kSplitF16 / kSplitBF16 of the current split
    uint64_t gen = 1;            // bumped whenever the tiles are written
    uint64_t split_gen = 0;      // gen the split was made from
    int64_t lvl_off[spamm::kMaxLevels] = {};
    int32_t lvl_m[spamm::kMaxLevels] = {};
    int64_t norms_total = 0;
    spamm::ProductScratch* ps = nullptr;
    spamm_alloc_fn alloc = nullptr;
    spamm_dealloc_fn dealloc = nullptr;
    void* actx = nullptr;
    hipStream_t last_stream = nullptr;
    int device = 0;
};

namespace spamm {

// error plumbing -------------------------------------------------------------
spamm_status set_error(spamm_status s, const std::string& msg);
spamm_status hip_error(hipError_t e, const char* what);

#define SPAMM_HIP(call)                                          \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return ::spamm::hip_error(e_, #call); \
    } while (0)

// allocation ------------------------------------------------------------------
// The allocator pair an object was created with (the hook of
// spamm_set_allocator at that time; null functions: hipMalloc / hipFree).
struct Allocator {
    spamm_alloc_fn alloc = nullptr;
    spamm_dealloc_fn dealloc = nullptr;
    void* ctx = nullptr;
};
Allocator current_allocator();
// Stream-ordered allocation and release through an allocator pair.
void* raw_alloc(const Allocator& a, size_t bytes, hipStream_t s);
void raw_free(const Allocator& a, void* p, hipStream_t s);
void* dev_alloc(spamm_matrix* owner, size_t bytes, hipStream_t s);
void dev_free(spamm_matrix* owner, void* p, hipStream_t s);
int num_cus();

// Tile layout of a handle (see TileGeo).
inline TileGeo tile_geo(const spamm_matrix* M) {
    TileGeo g;
    g.b = M->b;
    g.pad_ = 0;
    if (M->view) {
        g.si = (int64_t)M->b * M->ld;
        g.sk = M->b;
        g.ld = M->ld;
    } else {
        g.si = M->nb * M->b * (int64_t)M->b;
        g.sk = (int64_t)M->b * M->b;
        g.ld = M->b;
    }
    return g;
}

// launchers (norms.hip) ---------------------------------------------------------
// split_kind >= 0 (FP32 input, M->split allocated): the same pass also writes
// the split 16-bit tiles of that kind.
hipError_t launch_pack_norm(const void* a, int64_t n, int64_t lda, spamm_dtype dt, spamm_matrix* M,
                            int split_kind, hipStream_t s);
hipError_t launch_upper_norms(spamm_matrix* M, hipStream_t s, const int* active);
// The tiers above the leaves are formed when something reads them: builds
// and single products write the leaf norms only, and ensure_tiers enqueues
// the upper tiers of M on s (a no-op when they are current).
spamm_status ensure_tiers(const spamm_matrix* M, hipStream_t s, const int* active = nullptr);

// Batched builds and result pyramids (norms.hip).
struct PackDesc {
    const void* a;            // dense row-major input
    int64_t n, lda, nb, nstrips;
    int64_t wave_base;        // first global wave of this matrix
    void* tiles;              // NULL: norms only (a view)
    double* S0;               // leaf tier of the pyramid
    int8_t* texp;
    int32_t vec, pad_;
};
struct NormTable {
    double* norms;
    int64_t off[kMaxLevels];
    int32_t m[kMaxLevels];
    int32_t L, pad_;
};
PackDesc pack_desc(const void* a, int64_t n, int64_t lda, spamm_matrix* M, int64_t wave_base);
NormTable norm_table(const spamm_matrix* M);
hipError_t launch_pack_norm_batched(const PackDesc* d_pd, int count, int64_t waves, spamm_dtype dt, int b,
                                    hipStream_t s);
hipError_t launch_upper_norms_batched(spamm_matrix* const* M, int count, const NormTable* d_tab, hipStream_t s);
hipError_t launch_to_dense(const spamm_matrix* M, void* out, int64_t ldo, hipStream_t s);
hipError_t launch_diff_norms(const spamm_matrix* X, const spamm_matrix* Y, double* d_out, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, int64_t count, uint64_t v, hipStream_t s);

// split.hip: hi/lo 16-bit copies of an FP32 handle's tiles into M->split
hipError_t launch_split(const spamm_matrix* M, int kind, const int* active, hipStream_t s);

// launchers (cull.hip) ----------------------------------------------------------
struct Sp2State;
struct CullPlan {
    int count;              // products in the batch
    int Lmax;               // highest tier among the products
    int64_t front_cap;      // capacity of each frontier buffer (keys)
    int64_t mask_words;     // total leaf-bitmask words
    unsigned long long* nonempty = nullptr;  // per-product non-empty tile counters (zeroed with the rest)
    int flat_start = 0;     // single product, flat threshold: enumerate tier flat_start (>= 1) directly
    int flat_m = 0;         //   its size m; the tiers above it are not visited (nor counted)
    int leaf_direct = 0;    // single product, flat threshold: test every leaf triple, no tiers visited
    int64_t leaf_nb = 0;    //   (nb of the product; the leaf tier's kept count is still counted)
    uint32_t* sp2_list = nullptr;   // direct leaf pass of an SP2 step: also list the C tiles to write
    Sp2State* sp2_state = nullptr;  //   (and their count); the counters are kept at zero by the step
    bool skip_prep = false;         //   finalize, so no zeroing launch precedes the pass
    bool uncounted = false;         // direct leaf pass whose counters nobody reads (no zeroing, no counts)
};
hipError_t launch_cull_ex(const ProdDesc* d_desc, const CullPlan& plan, uint64_t* mask, uint64_t* front0,
                          uint64_t* front1, DevCounters* ctr, int want_bound, const int* active,
                          const int64_t* tier_items, hipStream_t s);
// Batch of flat-threshold products without statistics: every leaf triple
// tested, one block per (product, tile row, 64 tiles); d_blk_off[m] is the
// first block of product m, blocks the total.  Writes every mask word.
hipError_t launch_cull_leaf_batched(const ProdDesc* d_desc, int nprod, const int64_t* d_blk_off, int64_t blocks,
                                   hipStream_t s);
hipError_t launch_task_keys(const ProdDesc* d_desc, int64_t nb, int W, const uint64_t* mask,
                            uint64_t* keys_out, unsigned long long* count, int64_t cap, hipStream_t s);

// launchers (leaf.hip) ----------------------------------------------------------
struct LeafPlan {
    int count;
    int64_t total_tiles;    // sum over products of nb^2
    int b;
    spamm_leaf_prec prec;
    bool c_f64;
    int sp2;                // 1: fuse the TC2 update into the epilogue
    const int* d_branch;    // SP2: device branch flag (0: X^2, 1: 2X - X^2)
    const int* d_active;    // SP2: device flag, 0 = skip (converged)
    const uint32_t* order = nullptr;       // persistent launch: tile order (NULL = identity)
    unsigned long long* queue = nullptr;   // persistent launch: zeroed queue counter (NULL = static grid)
    bool presplit = false;                 // 16-bit leaves: every operand has current split tiles
    const uint32_t* list = nullptr;        // C tiles to visit (persistent launch over the list)
    const unsigned* list_count = nullptr;  //   and their device-side count
    unsigned* list_queue = nullptr;        //   zeroed queue counter: blocks pull list positions (NULL: static stride)
};
hipError_t launch_lpt_order(const ProdDesc* d_desc, int nprod, int64_t total, int maxc, uint32_t* counts,
                            uint32_t* hist, uint32_t* offs, uint32_t* order, unsigned long long* queue,
                            hipStream_t s);
hipError_t launch_clear_masks(const ProdDesc* d_desc, int nprod, hipStream_t s);
hipError_t launch_tile_list(const ProdDesc* d_desc, int nprod, int64_t total, uint32_t* list, unsigned* count,
                            unsigned* queue, hipStream_t s);
hipError_t launch_leaf_typed(const ProdDesc* d_desc, const LeafPlan& plan, bool a_f64, hipStream_t s);

// SP2 device state (sp2.hip): the branch/active flags read by the product
// kernels, the per-step log and the stopping parameters.
struct Sp2State {
    int branch;          // 0: X <- X^2, 1: X <- 2X - X^2 (for the current step)
    int active;          // 0 once a stop rule fired
    int iter, converged, stagnated, result_step, max_iter, pad_;
    double cur_trace;    // tr(X_iter)
    double n_occ, tol;
    double eps_min, eps_max;
    double trace[SPAMM_SP2_MAX_ITER];
    double idem[SPAMM_SP2_MAX_ITER];
    int br[SPAMM_SP2_MAX_ITER];
    unsigned long long tasks[SPAMM_SP2_MAX_ITER];
    unsigned list_count;  // C tiles of the current step that the leaf launch visits
    unsigned fin_ticket;  // blocks of the per-step finalize that are done (reset by the last)
    double fin_bsum[64];  // their partial sums
    unsigned sym_bad;     // symmetric SP2: set when H is not exactly symmetric
    unsigned pad3_;
};
hipError_t launch_gershgorin(const spamm_matrix* H, double* lo, double* hi, Sp2State* st, hipStream_t s);
hipError_t launch_sp2_init(const spamm_matrix* H, spamm_matrix* X, double* part, Sp2State* st, hipStream_t s);
hipError_t launch_sp2_finalize(const double* part, int64_t nb, unsigned long long* survivors0, Sp2State* st,
                               int m, hipStream_t s);
hipError_t launch_energy(const spamm_matrix* P, const spamm_matrix* H, double* tile_part, double* out,
                         hipStream_t s);
// Dropping scheme: zero the tiles of X with S < tau2 (norm 0, exponent -128,
// diagonal trace partial 0); skipped once the SP2 state is inactive.
hipError_t launch_sp2_drop(spamm_matrix* X, double* part, double tau2, const int* active, hipStream_t s);
hipError_t launch_sp2_tiles(const ProdDesc* d_desc, int64_t nb, uint32_t* list, Sp2State* st, const int* active,
                            hipStream_t s);
hipError_t launch_check_symmetric(const spamm_matrix* H, unsigned* flag, hipStream_t s);

// api.hip: cull + leaf products + result pyramid of one product, enqueued
spamm_status enqueue_product(const spamm_matrix* A, const spamm_matrix* B, spamm_matrix* C, double tau,
                             spamm_leaf_prec prec, hipStream_t s, int want_bound, int sp2, const int* d_branch,
                             const int* d_active, ProdDesc* d_desc_override, uint32_t* sp2_list = nullptr,
                             Sp2State* sp2_state = nullptr, int depth_tau = 0, bool count_tasks = false);
// C ~= A B (flat tau) with only the kept-product count as a statistic: no
// per-tier survivors or culled bound, so the direct leaf pass serves it.
// Synchronises the stream.  *C as for spamm_multiply.
spamm_status multiply_count(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec,
                            hipStream_t s, spamm_matrix** C, int64_t* tasks);

}  // namespace spamm
