// extern "C" entry points of libspamm (declared in include/spamm.h).
//
// Host-side validation happens before anything is enqueued; device-side
// conditions are reported by syncing calls (a product's capacity flag in its
// counters; a non-finite operand by its root norm, which an inf or NaN
// anywhere in the matrix makes non-finite).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spamm_internal.hpp"

namespace spamm {

namespace {
thread_local std::string g_err;
spamm_alloc_fn g_alloc = nullptr;
spamm_dealloc_fn g_dealloc = nullptr;
void* g_actx = nullptr;
std::mutex g_mu;
thread_local hipEvent_t* t_phase = nullptr;  // set by spamm_multiply_timed
}  // namespace

spamm_status set_error(spamm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

spamm_status hip_error(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SPAMM_ENOMEM : SPAMM_EHIP;
}

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_mu);
    Allocator a;
    a.alloc = g_alloc;
    a.dealloc = g_dealloc;
    a.ctx = g_actx;
    return a;
}

void* raw_alloc(const Allocator& a, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (a.alloc) return a.alloc(bytes, (void*)s, a.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void raw_free(const Allocator& a, void* p, hipStream_t s) {
    if (!p) return;
    if (a.dealloc) a.dealloc(p, (void*)s, a.ctx);
    else (void)hipFree(p);
}

void* dev_alloc(spamm_matrix* owner, size_t bytes, hipStream_t s) {
    Allocator a;
    a.alloc = owner->alloc;
    a.dealloc = owner->dealloc;
    a.ctx = owner->actx;
    return raw_alloc(a, bytes, s);
}

void dev_free(spamm_matrix* owner, void* p, hipStream_t s) {
    Allocator a;
    a.alloc = owner->alloc;
    a.dealloc = owner->dealloc;
    a.ctx = owner->actx;
    raw_free(a, p, s);
}

int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool leaf_ok(int32_t b) { return b == 32 || b == 64 || b == 128; }

// Tier shapes m_0 = nb, m_{l+1} = ceil(m_l / 2) ... m_L = 1.
void tier_shapes(int64_t nb, int32_t& L, int32_t* m, int64_t* off, int64_t& total) {
    L = 0;
    int64_t mm = nb;
    total = 0;
    for (int l = 0;; ++l) {
        m[l] = (int32_t)mm;
        off[l] = total;
        total += mm * mm;
        if (mm == 1) {
            L = l;
            break;
        }
        mm = ceil_div(mm, 2);
    }
}

spamm_matrix* new_handle(int64_t n, int32_t b, spamm_dtype dt) {
    auto* M = new spamm_matrix();
    M->n = n;
    M->b = b;
    M->nb = ceil_div(n, b);
    M->dt = dt;
    M->elem = dt == SPAMM_F64 ? 8 : 4;
    tier_shapes(M->nb, M->L, M->lvl_m, M->lvl_off, M->norms_total);
    const Allocator a = current_allocator();
    M->alloc = a.alloc;
    M->dealloc = a.dealloc;
    M->actx = a.ctx;
    (void)hipGetDevice(&M->device);
    return M;
}

void release_scratch(spamm_matrix* M) {
    if (!M->ps) return;
    ProductScratch* ps = M->ps;
    dev_free(M, ps->mask, M->last_stream);
    dev_free(M, ps->front[0], M->last_stream);
    dev_free(M, ps->front[1], M->last_stream);
    dev_free(M, ps->ctr, M->last_stream);
    dev_free(M, ps->desc, M->last_stream);
    dev_free(M, ps->sp2_part, M->last_stream);
    delete ps;
    M->ps = nullptr;
}

void release(spamm_matrix* M) {
    if (!M) return;
    if (M->last_stream) (void)hipStreamSynchronize(M->last_stream);
    release_scratch(M);
    if (!M->view) dev_free(M, M->tiles, M->last_stream);
    dev_free(M, M->norms, M->last_stream);
    dev_free(M, M->texp, M->last_stream);
    dev_free(M, M->split, M->last_stream);
    delete M;
}

// Device storage of a handle: tiles (not for a view), norm pyramid (+ tier
// tables + status word at its tail) and per-tile exponents.
spamm_status alloc_storage(spamm_matrix* M, hipStream_t s) {
    const size_t tiles = (size_t)(M->nb * M->nb) * M->b * M->b * M->elem;
    if (!M->view) M->tiles = dev_alloc(M, tiles, s);
    const size_t nbytes = (size_t)M->norms_total * 8 + kMaxLevels * 8 + kMaxLevels * 4 + 64;
    M->norms = (double*)dev_alloc(M, nbytes, s);
    M->texp = (int8_t*)dev_alloc(M, (size_t)(M->nb * M->nb), s);
    if (!M->tiles || !M->norms || !M->texp) return set_error(SPAMM_ENOMEM, "device allocation failed");
    // exponent 0 = "tile not known to be zero": products skip rewriting only
    // tiles a previous write left at zero (exponent -128)
    SPAMM_HIP(hipMemsetAsync(M->texp, 0, (size_t)(M->nb * M->nb), s));
    int64_t* off = reinterpret_cast<int64_t*>(M->norms + M->norms_total);
    int* mm = reinterpret_cast<int*>(off + kMaxLevels);
    SPAMM_HIP(hipMemcpyAsync(off, M->lvl_off, sizeof(int64_t) * kMaxLevels, hipMemcpyHostToDevice, s));
    SPAMM_HIP(hipMemcpyAsync(mm, M->lvl_m, sizeof(int32_t) * kMaxLevels, hipMemcpyHostToDevice, s));
    return SPAMM_OK;
}

}  // namespace

spamm_status ensure_tiers(const spamm_matrix* Mc, hipStream_t s, const int* active) {
    auto* M = const_cast<spamm_matrix*>(Mc);  // the upper tiers are a cache of the leaf norms
    if (M->tiers_valid) return SPAMM_OK;
    SPAMM_HIP(launch_upper_norms(M, s, active));
    M->tiers_valid = true;
    return SPAMM_OK;
}

namespace {

// The squared Frobenius norm of the whole matrix (the root of its pyramid)
// is finite iff every element is: x*x of an inf or NaN is inf or NaN, and
// FP64 sums of FP32 squares cannot overflow.  Call after the stream syncs.
spamm_status check_finite(const spamm_matrix* M, hipStream_t s, const char* what) {
    SPAMM_HIP(hipStreamSynchronize(s));
    double root = 0.0;
    SPAMM_HIP(hipMemcpy(&root, M->norms + M->lvl_off[M->L], sizeof root, hipMemcpyDeviceToHost));
    if (!std::isfinite(root)) return set_error(SPAMM_ENONFINITE, std::string("non-finite value in ") + what);
    return SPAMM_OK;
}

// Product scratch owned by the result handle.
spamm_status ensure_scratch(spamm_matrix* C, hipStream_t s) {
    if (C->ps) return SPAMM_OK;
    auto* ps = new ProductScratch();
    C->ps = ps;
    const int64_t nb = C->nb;
    const int W = (int)ceil_div(nb, 64);
    ps->mask = (uint64_t*)dev_alloc(C, (size_t)(nb * nb * W) * 8, s);
    int64_t cap = 1;
    if (C->L >= 2) cap = (int64_t)C->lvl_m[1] * C->lvl_m[1] * C->lvl_m[1];
    ps->front_cap = cap;
    ps->front[0] = (uint64_t*)dev_alloc(C, (size_t)cap * 8, s);
    ps->front[1] = (uint64_t*)dev_alloc(C, (size_t)cap * 8, s);
    ps->ctr = (DevCounters*)dev_alloc(C, sizeof(DevCounters) + 16 * kMaxBatch, s);
    ps->desc = (ProdDesc*)dev_alloc(C, sizeof(ProdDesc), s);
    if (!ps->mask || !ps->front[0] || !ps->front[1] || !ps->ctr || !ps->desc)
        return set_error(SPAMM_ENOMEM, "device allocation of product scratch failed");
    return SPAMM_OK;
}

// nonempty-tile counters live right after the DevCounters block
unsigned long long* nonempty_ctr(DevCounters* ctr) {
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(ctr) + sizeof(DevCounters));
}

ProdDesc make_desc(const spamm_matrix* A, const spamm_matrix* B, spamm_matrix* C, double tau) {
    ProdDesc d;
    std::memset(&d, 0, sizeof d);
    d.A = A->tiles;
    d.B = B->tiles;
    d.C = C->tiles;
    d.SA = A->norms;
    d.SB = B->norms;
    d.SC = C->norms;
    d.eA = A->texp;
    d.eB = B->texp;
    d.eC = C->texp;
    d.ga = tile_geo(A);
    d.gb = tile_geo(B);
    d.A16 = A->split;  // read only when current (LeafPlan::presplit)
    d.B16 = B->split;
    d.mask = C->ps->mask;
    d.nonempty = nonempty_ctr(C->ps->ctr);
    for (int l = 0; l < kMaxLevels; ++l) {
        d.lvl_off[l] = C->lvl_off[l];
        d.lvl_m[l] = C->lvl_m[l];
    }
    d.tile_base = 0;
    d.tau2 = tau * tau;
    d.nb = (int32_t)C->nb;
    d.L = C->L;
    d.W = (int32_t)ceil_div(C->nb, 64);
    d.a_f64 = A->dt == SPAMM_F64;
    d.b_f64 = B->dt == SPAMM_F64;
    return d;
}

spamm_status check_operands(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec) {
    if (!A || !B) return set_error(SPAMM_EINVAL, "null operand");
    if (A->n != B->n || A->b != B->b) return set_error(SPAMM_EINVAL, "operands differ in n or leaf size");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return set_error(SPAMM_EINVAL, "tau must be finite and >= 0");
    if (tau > 0.0 && tau < 1e-150) return set_error(SPAMM_EINVAL, "0 < tau < 1e-150: tau^2 would underflow");
    if ((int)prec < 0 || (int)prec > 5) return set_error(SPAMM_EINVAL, "unknown leaf precision");
    if (prec != SPAMM_LEAF_F64 && (A->dt != SPAMM_F32 || B->dt != SPAMM_F32))
        return set_error(SPAMM_EUNSUPPORTED, "leaf precisions below FP64 take FP32 operand tiles");
    if (prec == SPAMM_LEAF_F64 && A->dt != B->dt)
        return set_error(SPAMM_EUNSUPPORTED, "FP64 leaves take operands of one element type");
    // the leaf kernels step between operand tiles with 32-bit byte strides
    for (const spamm_matrix* M : {A, B}) {
        const TileGeo g = tile_geo(M);
        if (std::max(g.si, g.sk) * (int64_t)M->elem > (int64_t)UINT32_MAX)
            return set_error(SPAMM_EUNSUPPORTED, "an operand tile row exceeds 4 GiB");
    }
    return SPAMM_OK;
}

// Host upper bound of the nodes stored at each tier (for grid sizing).
void tier_items(const spamm_matrix* C, int64_t cap, int64_t* items) {
    for (int l = 0; l < kMaxLevels; ++l) items[l] = 0;
    for (int l = 1; l <= C->L; ++l) {
        const int64_t m = C->lvl_m[l];
        items[l] = std::min<int64_t>(m * m * m, cap);
    }
    items[C->L] = 0;  // the root enters as a virtual item
}

spamm_status read_stats(spamm_matrix* C, hipStream_t s, spamm_stats* st, double tau) {
    SPAMM_HIP(hipStreamSynchronize(s));
    DevCounters h;
    unsigned long long ne = 0;
    SPAMM_HIP(hipMemcpy(&h, C->ps->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost));
    SPAMM_HIP(hipMemcpy(&ne, nonempty_ctr(C->ps->ctr), sizeof ne, hipMemcpyDeviceToHost));
    std::memset(st, 0, sizeof *st);
    st->n = C->n;
    st->leaf = C->b;
    st->levels = C->L;
    st->nb = C->nb;
    for (int l = 0; l <= C->L && l < kMaxLevels; ++l) st->survivors[l] = (int64_t)h.survivors[0][l];
    st->tasks = st->survivors[0];
    st->nonempty_tiles = (int64_t)ne;
    st->flops = 2.0 * C->b * (double)C->b * C->b * (double)st->tasks;
    st->culled_bound = h.culled_bound[0];
    (void)tau;
    if (h.status & kDevCapacity) return set_error(SPAMM_ECAPACITY, "frontier capacity exceeded");
    return SPAMM_OK;
}

// Split 16-bit tiles a leaf precision reads (-1: none).
int split_kind(spamm_leaf_prec p) {
    if (p == SPAMM_LEAF_F16 || p == SPAMM_LEAF_F16X3) return kSplitF16;
    if (p == SPAMM_LEAF_BF16 || p == SPAMM_LEAF_BF16X3) return kSplitBF16;
    return -1;
}

}  // namespace

// Allocate M's split tiles if needed (allocation only: safe before a capture).
static spamm_status alloc_split(const spamm_matrix* Mc, hipStream_t s) {
    auto* M = const_cast<spamm_matrix*>(Mc);  // the split is a cache of the tiles
    if (M->split) return SPAMM_OK;
    M->split = (uint16_t*)dev_alloc(M, (size_t)(M->nb * M->nb) * M->b * M->b * 2 * sizeof(uint16_t), s);
    if (!M->split) return set_error(SPAMM_ENOMEM, "device allocation of split tiles failed");
    M->split_gen = 0;
    return SPAMM_OK;
}

// M's split tiles hold the split of kind `kind` of its current tiles.
static bool split_current(const spamm_matrix* M, int kind) {
    return kind >= 0 && M->split && M->split_kind == kind && M->split_gen == M->gen;
}

// Shared by multiply and SP2: cull + leaf products + C pyramid, all enqueued.
// want_bound: 0 = no statistics (a flat product may test its leaf triples in
// one pass); 1 = statistics (the descent from the root, counts and the
// culled-node bound); 2 = the descent from the root without the bound.
spamm_status enqueue_product(const spamm_matrix* A, const spamm_matrix* B, spamm_matrix* C, double tau,
                             spamm_leaf_prec prec, hipStream_t s, int want_bound, int sp2, const int* d_branch,
                             const int* d_active, ProdDesc* d_desc_override, uint32_t* sp2_list,
                             Sp2State* sp2_state, int depth_tau, bool count_tasks) {
    ProductScratch* ps = C->ps;
    ProdDesc* d_desc = d_desc_override;
    // 16-bit leaves read the operands' split tiles when both are current
    // (spamm_build_ex, or SP2, which maintains them); otherwise they split
    // the FP32 tiles on the fly
    const int kind = split_kind(prec);
    const bool presplit = split_current(A, kind) && split_current(B, kind);
    // a flat threshold without per-tier statistics starts below the root
    // (L >= 2); up to 2^27 leaf triples it tests every one in a single pass.
    // Outside SP2 and without statistics, nothing reads that pass's counters
    // or the count of non-empty C tiles, and no kernel updates them.
    const bool flat = !depth_tau && !want_bound && C->L >= 2;
    const bool direct = flat && C->nb * C->nb * C->nb <= ((int64_t)1 << 27);
    const bool uncounted = direct && !sp2_list && !sp2 && !count_tasks;
    C->gen++;
    if (!d_desc) {
        ProdDesc d = make_desc(A, B, C, tau);
        d.depth_tau = depth_tau;
        if (uncounted) d.nonempty = nullptr;
        if (!ps->desc_valid || std::memcmp(&d, &ps->host_desc, sizeof d) != 0) {
            ps->host_desc = d;
            SPAMM_HIP(hipMemcpyAsync(ps->desc, &ps->host_desc, sizeof(ProdDesc), hipMemcpyHostToDevice, s));
            ps->desc_valid = true;
        }
        d_desc = ps->desc;
    }
    CullPlan cp;
    cp.count = 1;
    cp.Lmax = C->L;
    cp.front_cap = ps->front_cap;
    cp.mask_words = C->nb * C->nb * ceil_div(C->nb, 64);
    cp.nonempty = nonempty_ctr(ps->ctr);
    if (flat) {
        // flat threshold, no per-tier statistics: start at the first tier of
        // at most 64^3 nodes (the tiers above are implied by the flat rule);
        // with L >= 2 that tier lies below the root, which the tier passes
        // then never expand again
        int fs = 1;
        while (fs < C->L && C->lvl_m[fs] > 64) ++fs;
        cp.flat_start = fs;
        cp.flat_m = C->lvl_m[fs];
        // up to 2^27 leaf triples, testing every one in a single pass (no
        // frontier, no atomics per triple) beats the descent
        if (direct) {
            cp.leaf_direct = 1;
            cp.leaf_nb = C->nb;
            if (sp2_list) {
                // an SP2 step: the pass also lists the tiles to write, and
                // the step's finalize leaves the counters at zero
                cp.sp2_list = sp2_list;
                cp.sp2_state = sp2_state;
                cp.skip_prep = true;
            } else if (uncounted) {
                // a product without statistics: its counters are read by
                // nothing (statistics take the full descent, which zeroes them)
                cp.skip_prep = true;
                cp.uncounted = true;
            }
        }
    }
    if (!cp.leaf_direct) {
        // the descent reads the operands' upper tiers
        spamm_status r = ensure_tiers(A, s, d_active);
        if (r == SPAMM_OK && B != A) r = ensure_tiers(B, s, d_active);
        if (r != SPAMM_OK) return r;
    }
    int64_t items[kMaxLevels];
    tier_items(C, ps->front_cap, items);
    if (t_phase) SPAMM_HIP(hipEventRecord(t_phase[0], s));
    SPAMM_HIP(launch_cull_ex(d_desc, cp, ps->mask, ps->front[0], ps->front[1], ps->ctr, want_bound == 1, d_active,
                             items, s));
    LeafPlan lp;
    lp.count = 1;
    lp.total_tiles = C->nb * C->nb;
    lp.b = C->b;
    lp.prec = prec;
    lp.c_f64 = C->dt == SPAMM_F64;
    lp.sp2 = sp2;
    lp.d_branch = d_branch;
    lp.d_active = d_active;
    lp.presplit = presplit;
    if (sp2_list) {
        // SP2: the leaf launch visits only the C tiles that need a write
        if (!cp.sp2_list) SPAMM_HIP(launch_sp2_tiles(d_desc, C->nb, sp2_list, sp2_state, d_active, s));
        lp.list = sp2_list;
        lp.list_count = &sp2_state->list_count;
        // (static stride: a step lists a few tiles per block, too few for a
        // queue's grabs to pay for themselves)
    }
    if (t_phase) SPAMM_HIP(hipEventRecord(t_phase[1], s));
    SPAMM_HIP(launch_leaf_typed(d_desc, lp, A->dt == SPAMM_F64, s));
    if (t_phase) SPAMM_HIP(hipEventRecord(t_phase[2], s));
    // the leaf epilogue wrote C's leaf norms; its upper tiers follow on demand
    C->tiers_valid = false;
    if (t_phase) SPAMM_HIP(hipEventRecord(t_phase[3], s));
    return SPAMM_OK;
}

}  // namespace spamm

using namespace spamm;

namespace {

// A view reads its tiles from the caller's array with 32-bit buffer offsets,
// 16-byte loads and no padding.
spamm_status check_view(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf) {
    const int64_t elem = dt == SPAMM_F64 ? 8 : 4;
    if (n % leaf != 0) return set_error(SPAMM_EINVAL, "a view needs n to be a multiple of the leaf size");
    if ((uintptr_t)dev_a % 16 != 0 || (lda * elem) % 16 != 0)
        return set_error(SPAMM_EINVAL, "a view needs a 16-byte aligned array and row pitch");
    if ((int64_t)leaf * lda * elem > (int64_t)INT32_MAX)
        return set_error(SPAMM_EINVAL, "a view needs leaf * lda * element size < 2^31 bytes");
    return SPAMM_OK;
}

spamm_status build_single(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                          spamm_leaf_prec prec, bool view, void* stream, spamm_matrix** out) {
    if (!out) return set_error(SPAMM_EINVAL, "out is null");
    if (!dev_a) return set_error(SPAMM_EINVAL, "dev_a is null");
    if (n < 1 || lda < n) return set_error(SPAMM_EINVAL, "need n >= 1 and lda >= n");
    if (dt != SPAMM_F32 && dt != SPAMM_F64) return set_error(SPAMM_EINVAL, "unknown dtype");
    if (!leaf_ok(leaf)) return set_error(SPAMM_EINVAL, "leaf must be 32, 64 or 128");
    if ((int)prec < 0 || (int)prec > 5) return set_error(SPAMM_EINVAL, "unknown leaf precision");
    if (ceil_div(n, leaf) > kMaxNb) return set_error(SPAMM_EINVAL, "n / leaf exceeds 2^19 leaves");
    if (view) {
        spamm_status v = check_view(dev_a, n, lda, dt, leaf);
        if (v != SPAMM_OK) return v;
    }
    const int kind = split_kind(prec);
    if (kind >= 0 && dt != SPAMM_F32)
        return set_error(SPAMM_EUNSUPPORTED, "16-bit leaf precisions take FP32 tiles");
    hipStream_t s = (hipStream_t)stream;
    spamm_matrix* M = *out;
    const bool fresh = M == nullptr;
    spamm_status st = SPAMM_OK;
    if (!fresh) {
        if (M->n != n || M->b != leaf || M->dt != dt)
            return set_error(SPAMM_EINVAL, "existing handle differs in n, leaf or dtype");
        if (M->view != view)
            return set_error(SPAMM_EINVAL, view ? "existing handle owns packed tiles (not a view)"
                                                : "existing handle is a view (spamm_build_view)");
    }
    if (fresh) {
        M = new_handle(n, leaf, dt);
        if (view) {
            M->view = true;
            M->tiles = const_cast<void*>(dev_a);
            M->ld = lda;
        }
        st = alloc_storage(M, s);
        if (st != SPAMM_OK) {
            release(M);
            return st;
        }
    } else if (view) {
        M->tiles = const_cast<void*>(dev_a);
        M->ld = lda;
    }
    if (kind >= 0 && (st = alloc_split(M, s)) != SPAMM_OK) {
        if (fresh) release(M);
        return st;
    }
    M->last_stream = s;
    M->gen++;
    hipError_t e = launch_pack_norm(dev_a, n, lda, dt, M, kind, s);
    M->tiers_valid = false;  // formed when read
    if (e != hipSuccess) {
        st = hip_error(e, "spamm_build kernels");
        if (fresh) release(M);
        return st;
    }
    if (kind >= 0) {
        M->split_kind = kind;
        M->split_gen = M->gen;
    }
    *out = M;
    return SPAMM_OK;
}

spamm_status build_batched(int32_t count, const void* const* dev_a, const int64_t* n, const int64_t* lda,
                           spamm_dtype dt, int32_t leaf, bool view, void* stream, spamm_matrix** out) {
    if (count < 1 || count > kMaxBatch) return set_error(SPAMM_EINVAL, "count outside [1, 128]");
    if (!dev_a || !n || !lda || !out) return set_error(SPAMM_EINVAL, "null argument");
    if (dt != SPAMM_F32 && dt != SPAMM_F64) return set_error(SPAMM_EINVAL, "unknown dtype");
    if (!leaf_ok(leaf)) return set_error(SPAMM_EINVAL, "leaf must be 32, 64 or 128");
    for (int m = 0; m < count; ++m) {
        if (!dev_a[m]) return set_error(SPAMM_EINVAL, "dev_a[m] is null");
        if (n[m] < 1 || lda[m] < n[m]) return set_error(SPAMM_EINVAL, "need n >= 1 and lda >= n");
        if (ceil_div(n[m], leaf) > kMaxNb) return set_error(SPAMM_EINVAL, "n / leaf exceeds 2^19 leaves");
        if (view) {
            spamm_status v = check_view(dev_a[m], n[m], lda[m], dt, leaf);
            if (v != SPAMM_OK) return v;
        }
        if (out[m] && (out[m]->n != n[m] || out[m]->b != leaf || out[m]->dt != dt))
            return set_error(SPAMM_EINVAL, "existing handle differs in n, leaf or dtype");
        if (out[m] && out[m]->view != view)
            return set_error(SPAMM_EINVAL, view ? "existing handle owns packed tiles (not a view)"
                                                : "existing handle is a view (spamm_build_view)");
        for (int q = 0; q < m; ++q)
            if (out[m] && out[m] == out[q]) return set_error(SPAMM_EINVAL, "out handles must be distinct");
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<spamm_matrix*> M(count, nullptr);
    std::vector<bool> fresh(count, false);
    auto release_fresh = [&]() {
        for (int m = 0; m < count; ++m)
            if (fresh[m] && M[m]) release(M[m]);
    };
    spamm_status st = SPAMM_OK;
    for (int m = 0; m < count && st == SPAMM_OK; ++m) {
        M[m] = out[m];
        if (!M[m]) {
            M[m] = new_handle(n[m], leaf, dt);
            fresh[m] = true;
            if (view) {
                M[m]->view = true;
                M[m]->tiles = const_cast<void*>(dev_a[m]);
                M[m]->ld = lda[m];
            }
            st = alloc_storage(M[m], s);
        }
    }
    if (st != SPAMM_OK) {
        release_fresh();
        return st;
    }
    static thread_local std::vector<PackDesc> hp;
    hp.resize(count);
    int64_t waves = 0;
    for (int m = 0; m < count; ++m) {
        M[m]->last_stream = s;
        M[m]->gen++;
        hp[m] = pack_desc(dev_a[m], n[m], lda[m], M[m], waves);
        waves += hp[m].nb * hp[m].nstrips;
    }
    const size_t bytes = sizeof(PackDesc) * count;
    char* ws = (char*)dev_alloc(M[0], bytes, s);
    if (!ws) {
        release_fresh();
        return set_error(SPAMM_ENOMEM, "batch scratch allocation failed");
    }
    const PackDesc* d_pd = (const PackDesc*)ws;
    hipError_t e = hipMemcpyAsync(ws, hp.data(), sizeof(PackDesc) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_pack_norm_batched(d_pd, count, waves, dt, leaf, s);
    // upper tiers when first read (a batch that descends forms the missing
    // ones of all its operands in one launch per tier)
    for (int m = 0; m < count; ++m) M[m]->tiers_valid = false;
    dev_free(M[0], ws, s);
    if (e != hipSuccess) {
        st = hip_error(e, "spamm_build_batched kernels");
        release_fresh();
        return st;
    }
    // a rebuilt view reads the new array
    for (int m = 0; m < count; ++m) {
        if (view) {
            M[m]->tiles = const_cast<void*>(dev_a[m]);
            M[m]->ld = lda[m];
        }
        out[m] = M[m];
    }
    return SPAMM_OK;
}

}  // namespace

extern "C" {

spamm_status spamm_build_ex(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                            spamm_leaf_prec prec, void* stream, spamm_matrix** out) {
    return build_single(dev_a, n, lda, dt, leaf, prec, false, stream, out);
}

spamm_status spamm_build_view(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                              void* stream, spamm_matrix** out) {
    return build_single(dev_a, n, lda, dt, leaf, dt == SPAMM_F64 ? SPAMM_LEAF_F64 : SPAMM_LEAF_F32, true, stream,
                        out);
}

spamm_status spamm_build_view_ex(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf,
                                 spamm_leaf_prec prec, void* stream, spamm_matrix** out) {
    return build_single(dev_a, n, lda, dt, leaf, prec, true, stream, out);
}

spamm_status spamm_build_batched(int32_t count, const void* const* dev_a, const int64_t* n, const int64_t* lda,
                                 spamm_dtype dt, int32_t leaf, void* stream, spamm_matrix** out) {
    return build_batched(count, dev_a, n, lda, dt, leaf, false, stream, out);
}

spamm_status spamm_build_view_batched(int32_t count, const void* const* dev_a, const int64_t* n,
                                      const int64_t* lda, spamm_dtype dt, int32_t leaf, void* stream,
                                      spamm_matrix** out) {
    return build_batched(count, dev_a, n, lda, dt, leaf, true, stream, out);
}

spamm_status spamm_build(const void* dev_a, int64_t n, int64_t lda, spamm_dtype dt, int32_t leaf, void* stream,
                         spamm_matrix** out) {
    return spamm_build_ex(dev_a, n, lda, dt, leaf, dt == SPAMM_F64 ? SPAMM_LEAF_F64 : SPAMM_LEAF_F32, stream, out);
}

namespace {
// force_descent: the cull descends tier by tier from the root (the path a
// product with statistics takes) even without statistics
spamm_status multiply_impl(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec,
                           int32_t tau_schedule, void* stream, spamm_matrix** C, spamm_stats* st,
                           bool force_descent) {
    if (!C) return set_error(SPAMM_EINVAL, "C is null");
    if (tau_schedule != SPAMM_TAU_FLAT && tau_schedule != SPAMM_TAU_DEPTH_SCALED)
        return set_error(SPAMM_EINVAL, "unknown tau schedule");
    spamm_status v = check_operands(A, B, tau, prec);
    if (v != SPAMM_OK) return v;
    // every tier's tau^2 must stay a normal FP64 number: tau / 8^L >= 1e-150
    if (tau_schedule == SPAMM_TAU_DEPTH_SCALED && tau > 0.0 && !(std::ldexp(tau, -3 * A->L) >= 1e-150))
        return set_error(SPAMM_EINVAL, "depth-scaled schedule needs tau / 8^L >= 1e-150");
    const spamm_dtype cdt = prec == SPAMM_LEAF_F64 ? SPAMM_F64 : SPAMM_F32;
    spamm_matrix* Cm = *C;
    if (Cm) {
        if (Cm == A || Cm == B) return set_error(SPAMM_EINVAL, "C may not alias an operand");
        if (Cm->view) return set_error(SPAMM_EINVAL, "a view cannot receive a product");
        if (Cm->n != A->n || Cm->b != A->b || Cm->dt != cdt)
            return set_error(SPAMM_EINVAL, "existing C differs in n, leaf or result type");
    }
    hipStream_t s = (hipStream_t)stream;
    bool fresh = false;
    if (!Cm) {
        Cm = new_handle(A->n, A->b, cdt);
        fresh = true;
        spamm_status r = alloc_storage(Cm, s);
        if (r != SPAMM_OK) {
            release(Cm);
            return r;
        }
    }
    Cm->last_stream = s;
    spamm_status r = ensure_scratch(Cm, s);
    if (r == SPAMM_OK)
        r = enqueue_product(A, B, Cm, tau, prec, s, st != nullptr ? 1 : (force_descent ? 2 : 0), 0, nullptr,
                            nullptr, nullptr, nullptr, nullptr, tau_schedule == SPAMM_TAU_DEPTH_SCALED);
    if (r != SPAMM_OK) {
        if (fresh) release(Cm);
        return r;
    }
    *C = Cm;
    if (st) {
        r = read_stats(Cm, s, st, tau);
        if (r == SPAMM_OK) r = ensure_tiers(A, s);
        if (r == SPAMM_OK) r = ensure_tiers(B, s);
        if (r == SPAMM_OK) r = check_finite(A, s, "operand A");
        if (r == SPAMM_OK) r = check_finite(B, s, "operand B");
        return r;
    }
    return SPAMM_OK;
}

}  // namespace

spamm_status spamm_multiply_ex(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec,
                               int32_t tau_schedule, void* stream, spamm_matrix** C, spamm_stats* st) {
    return multiply_impl(A, B, tau, prec, tau_schedule, stream, C, st, false);
}

spamm_status spamm_multiply(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec,
                            void* stream, spamm_matrix** C, spamm_stats* st) {
    return spamm_multiply_ex(A, B, tau, prec, SPAMM_TAU_FLAT, stream, C, st);
}

spamm_status spamm_multiply_timed(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec,
                                  void* stream, spamm_matrix** C, spamm_timing* t) {
    return spamm_multiply_timed_ex(A, B, tau, prec, 0, stream, C, t);
}

spamm_status spamm_multiply_timed_ex(const spamm_matrix* A, const spamm_matrix* B, double tau,
                                     spamm_leaf_prec prec, int32_t flags, void* stream, spamm_matrix** C,
                                     spamm_timing* t) {
    if (!t) return set_error(SPAMM_EINVAL, "timing output is null");
    if (flags & ~SPAMM_TIMED_DESCENT) return set_error(SPAMM_EINVAL, "unknown timing flags");
    static thread_local hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (!ev[0])
        for (auto& e : ev) SPAMM_HIP(hipEventCreate(&e));
    t_phase = ev;
    spamm_status r = multiply_impl(A, B, tau, prec, SPAMM_TAU_FLAT, stream, C, nullptr,
                                   (flags & SPAMM_TIMED_DESCENT) != 0);
    t_phase = nullptr;
    if (r != SPAMM_OK) return r;
    SPAMM_HIP(hipEventSynchronize(ev[3]));
    float a = 0, b = 0, c = 0, d = 0;
    SPAMM_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
    SPAMM_HIP(hipEventElapsedTime(&b, ev[1], ev[2]));
    SPAMM_HIP(hipEventElapsedTime(&c, ev[2], ev[3]));
    SPAMM_HIP(hipEventElapsedTime(&d, ev[0], ev[3]));
    t->ms_cull = a;
    t->ms_leaf = b;
    t->ms_norms = c;
    t->ms_total = d;
    return SPAMM_OK;
}

spamm_status spamm_to_dense(const spamm_matrix* M, void* dev_out, int64_t ldo, void* stream) {
    if (!M || !dev_out) return set_error(SPAMM_EINVAL, "null argument");
    if (ldo < M->n) return set_error(SPAMM_EINVAL, "ldo < n");
    SPAMM_HIP(launch_to_dense(M, dev_out, ldo, (hipStream_t)stream));
    return SPAMM_OK;
}

spamm_status spamm_info(const spamm_matrix* M, int64_t* n, int32_t* leaf, spamm_dtype* dt, int32_t* levels) {
    if (!M) return set_error(SPAMM_EINVAL, "null handle");
    if (n) *n = M->n;
    if (leaf) *leaf = M->b;
    if (dt) *dt = M->dt;
    if (levels) *levels = M->L;
    return SPAMM_OK;
}

spamm_status spamm_norms(const spamm_matrix* M, int32_t level, double* host_out, int64_t cap, void* stream) {
    if (!M || !host_out) return set_error(SPAMM_EINVAL, "null argument");
    if (level < 0 || level > M->L) return set_error(SPAMM_EINVAL, "level out of range");
    const int64_t m = M->lvl_m[level];
    if (cap < m * m) return set_error(SPAMM_EINVAL, "host buffer too small");
    hipStream_t s = (hipStream_t)stream;
    spamm_status r = ensure_tiers(M, s);
    if (r != SPAMM_OK) return r;
    SPAMM_HIP(hipStreamSynchronize(s));
    SPAMM_HIP(hipMemcpy(host_out, M->norms + M->lvl_off[level], sizeof(double) * m * m, hipMemcpyDeviceToHost));
    return check_finite(M, s, "the matrix");
}

spamm_status spamm_task_list(const spamm_matrix* C, uint64_t* host_keys, int64_t cap, int64_t* count,
                             void* stream) {
    if (!C || !count) return set_error(SPAMM_EINVAL, "null argument");
    if (!C->ps) return set_error(SPAMM_EINVAL, "handle was not written by a product");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = C->nb;
    const int W = (int)ceil_div(nb, 64);
    std::vector<uint64_t> mask((size_t)(nb * nb * W));
    SPAMM_HIP(hipStreamSynchronize(s));
    SPAMM_HIP(hipMemcpy(mask.data(), C->ps->mask, mask.size() * 8, hipMemcpyDeviceToHost));
    int64_t t = 0;
    for (int64_t tile = 0; tile < nb * nb; ++tile)
        for (int w = 0; w < W; ++w) {
            uint64_t bits = mask[(size_t)(tile * W + w)];
            while (bits) {
                const int k = __builtin_ctzll(bits);
                bits &= bits - 1;
                if (host_keys && t < cap)
                    host_keys[t] = ((uint64_t)(tile / nb) << 42) | ((uint64_t)(tile % nb) << 21) | (uint64_t)(w * 64 + k);
                ++t;
            }
        }
    *count = t;
    return SPAMM_OK;
}

spamm_status spamm_diff_norms(const spamm_matrix* X, const spamm_matrix* Y, double* diff2, double* ref2,
                              void* stream) {
    if (!X || !Y || !diff2 || !ref2) return set_error(SPAMM_EINVAL, "null argument");
    if (X->n != Y->n) return set_error(SPAMM_EINVAL, "handles differ in n");
    hipStream_t s = (hipStream_t)stream;
    const Allocator al = current_allocator();
    double* d = (double*)raw_alloc(al, 2 * 1024 * sizeof(double), s);
    if (!d) return set_error(SPAMM_ENOMEM, "spamm_diff_norms workspace allocation failed");
    std::vector<double> h(2048);
    hipError_t e = launch_diff_norms(X, Y, d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, h.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    raw_free(al, d, s);
    if (e != hipSuccess) return hip_error(e, "spamm_diff_norms");
    double a = 0.0, b = 0.0;
    for (int i = 0; i < 1024; ++i) {
        a += h[2 * i];
        b += h[2 * i + 1];
    }
    *diff2 = a;
    *ref2 = b;
    return SPAMM_OK;
}

spamm_status spamm_set_allocator(spamm_alloc_fn alloc, spamm_dealloc_fn dealloc, void* ctx) {
    if ((alloc == nullptr) != (dealloc == nullptr))
        return set_error(SPAMM_EINVAL, "alloc and dealloc must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    g_alloc = alloc;
    g_dealloc = dealloc;
    g_actx = ctx;
    return SPAMM_OK;
}

void spamm_free(spamm_matrix* M) { release(M); }

const char* spamm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace spamm {
namespace {

// Batch scratch of spamm_multiply_batched_noalloc: one copy per device, held
// until the process ends.  In host code `scratch` is only a stand-in for the
// symbol; the device address comes from hipGetSymbolAddress, once per device,
// and is what kernels and copies receive.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

spamm_status static_scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return set_error(SPAMM_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(SPAMM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPAMM_OK;
}

// count products in one cull and one leaf launch.  fixed: the batch scratch
// is the device's static array (no allocation; every C[m] must already hold
// its product scratch, no statistics, the direct leaf pass only); otherwise
// it comes from the allocator and is released, stream-ordered, at the end.
spamm_status multiply_batched_impl(int32_t count, const spamm_matrix* const* A, const spamm_matrix* const* B,
                                   const double* tau, spamm_leaf_prec prec, const spamm_tune* tune, void* stream,
                                   spamm_matrix** C, spamm_stats* st, bool fixed) {
    if (count < 1 || count > kMaxBatch) return set_error(SPAMM_EINVAL, "count outside [1, 128]");
    if (!A || !B || !tau || !C) return set_error(SPAMM_EINVAL, "null argument");
    if (!A[0]) return set_error(SPAMM_EINVAL, "null operand");
    const int32_t b = A[0]->b;
    const int sched = tune ? tune->schedule : SPAMM_SCHED_LPT;
    if (sched != SPAMM_SCHED_STATIC && sched != SPAMM_SCHED_LPT && sched != SPAMM_SCHED_LIST)
        return set_error(SPAMM_EINVAL, "unknown schedule");
    if (tune && tune->leaf && tune->leaf != b) return set_error(SPAMM_EINVAL, "tune->leaf differs from the operands");
    const spamm_dtype cdt = prec == SPAMM_LEAF_F64 ? SPAMM_F64 : SPAMM_F32;
    int dev = 0;
    if (fixed) {
        if (st) return set_error(SPAMM_EINVAL, "the allocation-free product fills no statistics");
        hipError_t ge = hipGetDevice(&dev);
        if (ge != hipSuccess) return hip_error(ge, "hipGetDevice");
    }
    for (int m = 0; m < count; ++m) {
        if (fixed) {
            if (!C[m] || !C[m]->ps)
                return set_error(SPAMM_EINVAL, "the allocation-free product needs every C[m] to be a result handle "
                                               "that has received a product (its product scratch in place)");
            if (C[m]->device != dev) return set_error(SPAMM_EINVAL, "C[m] lives on another device than the current one");
        }
        spamm_status v = check_operands(A[m], B[m], tau[m], prec);
        if (v != SPAMM_OK) return v;
        if (A[m]->b != b) return set_error(SPAMM_EINVAL, "products of one batch share the leaf size");
        if (A[m]->dt != A[0]->dt) return set_error(SPAMM_EINVAL, "products of one batch share the operand type");
        if (C[m]) {
            if (C[m]->view) return set_error(SPAMM_EINVAL, "a view cannot receive a product");
            if (C[m]->n != A[m]->n || C[m]->b != b || C[m]->dt != cdt)
                return set_error(SPAMM_EINVAL, "existing C differs in n, leaf or result type");
            for (int q = 0; q < count; ++q)
                if (C[m] == A[q] || C[m] == B[q] || (q != m && C[m] == C[q]))
                    return set_error(SPAMM_EINVAL, "C handles must be distinct and not alias operands");
        }
    }
    hipStream_t s = (hipStream_t)stream;
    spamm_matrix* out[kMaxBatch] = {};
    bool fresh[kMaxBatch] = {};
    spamm_status r = SPAMM_OK;
    auto release_fresh = [&]() {
        for (int m = 0; m < count; ++m)
            if (fresh[m] && out[m]) release(out[m]);
    };
    for (int m = 0; m < count && r == SPAMM_OK; ++m) {
        out[m] = C[m];
        if (!out[m]) {
            out[m] = new_handle(A[m]->n, b, cdt);
            fresh[m] = true;
            r = alloc_storage(out[m], s);
        }
        if (r == SPAMM_OK) {
            out[m]->last_stream = s;
            r = ensure_scratch(out[m], s);
        }
    }
    if (r != SPAMM_OK) {
        release_fresh();
        return r;
    }
    // batch plan
    int64_t total = 0, cap = 1, items[kMaxLevels] = {};
    int Lmax = 0, maxc = 1;
    const int kind = split_kind(prec);
    bool presplit = kind >= 0;
    for (int m = 0; m < count; ++m) presplit = presplit && split_current(A[m], kind) && split_current(B[m], kind);
    static thread_local ProdDesc hd[kMaxBatch];
    for (int m = 0; m < count; ++m) {
        spamm_matrix* Cm = out[m];
        hd[m] = make_desc(A[m], B[m], Cm, tau[m]);
        hd[m].tile_base = total;
        total += Cm->nb * Cm->nb;
        Lmax = std::max(Lmax, Cm->L);
        maxc = std::max<int>(maxc, (int)Cm->nb);
        if (Cm->L >= 2) cap += (int64_t)Cm->lvl_m[1] * Cm->lvl_m[1] * Cm->lvl_m[1];
        for (int l = 1; l < Cm->L; ++l) items[l] += (int64_t)Cm->lvl_m[l] * Cm->lvl_m[l] * Cm->lvl_m[l];
    }
    for (int l = 0; l < kMaxLevels; ++l) items[l] = std::min(items[l], cap);
    // without statistics the flat rule needs no tier above the leaves: up to
    // 2^27 leaf triples in all, every triple is tested in one pass
    static thread_local int64_t hblk[kMaxBatch + 1];
    hblk[0] = 0;
    int64_t triples = 0;
    for (int m = 0; m < count; ++m) {
        const int64_t nbm = out[m]->nb;
        triples += nbm * nbm * nbm;
        hblk[m + 1] = hblk[m] + nbm * ceil_div(nbm, 64);
    }
    const bool direct = st == nullptr && triples <= ((int64_t)1 << 27);
    if (fixed && !direct)
        return set_error(SPAMM_ECAPACITY, "the allocation-free product takes at most 2^27 leaf triples in all "
                                          "(sum of nb^3 over the batch)");
    // the frontiers are read only by the descent
    const int64_t fcap = direct ? 0 : cap;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_desc = 0, o_f0 = al(sizeof(ProdDesc) * count), o_f1 = o_f0 + al((size_t)fcap * 8),
                 o_ctr = o_f1 + al((size_t)fcap * 8), o_cnt = o_ctr + al(sizeof(DevCounters) + 16 * kMaxBatch),
                 o_ord = o_cnt + al((size_t)total * 4), o_hist = o_ord + al((size_t)total * 4),
                 o_offs = o_hist + al((size_t)(maxc + 1) * 4), o_q = o_offs + al((size_t)(maxc + 1) * 4),
                 o_tab = o_q + 256, o_blk = o_tab + al(sizeof(NormTable) * 2 * count),
                 bytes = o_blk + al(sizeof(int64_t) * (count + 1));
    spamm_matrix* owner = out[0];
    char* ws = nullptr;
    if (fixed) {
        if (bytes > kStaticScratchBytes)
            return set_error(SPAMM_ECAPACITY, "batch plan exceeds the static scratch (16 MiB)");
        spamm_status r2 = static_scratch_ptr(dev, (void**)&ws);
        if (r2 != SPAMM_OK) return r2;
    } else {
        ws = (char*)dev_alloc(owner, bytes, s);
        if (!ws) {
            release_fresh();
            return set_error(SPAMM_ENOMEM, "batch scratch allocation failed");
        }
    }
    ProdDesc* d_desc = (ProdDesc*)(ws + o_desc);
    DevCounters* ctr = (DevCounters*)(ws + o_ctr);
    for (int m = 0; m < count; ++m) {
        // the non-empty tile counts are read only with statistics
        hd[m].nonempty = st ? nonempty_ctr(ctr) + m : nullptr;
        out[m]->ps->desc_valid = false;
        out[m]->gen++;
    }
    CullPlan cp;
    cp.count = count;
    cp.Lmax = Lmax;
    cp.front_cap = cap;
    cp.mask_words = 0;
    cp.nonempty = nonempty_ctr(ctr);
    LeafPlan lp;
    lp.count = count;
    lp.total_tiles = total;
    lp.b = b;
    lp.prec = prec;
    lp.c_f64 = cdt == SPAMM_F64;
    lp.sp2 = 0;
    lp.d_branch = nullptr;
    lp.d_active = nullptr;
    lp.presplit = presplit;
    if (sched == SPAMM_SCHED_LPT) {
        lp.order = (uint32_t*)(ws + o_ord);
        lp.queue = (unsigned long long*)(ws + o_q);
    } else if (sched == SPAMM_SCHED_LIST) {
        lp.list = (uint32_t*)(ws + o_ord);  // the order array holds the list
        lp.list_count = (unsigned*)(ws + o_q);
        lp.list_queue = (unsigned*)(ws + o_q + 64);
    }
    hipError_t e = hipMemcpyAsync(d_desc, hd, sizeof(ProdDesc) * count, hipMemcpyHostToDevice, s);
    if (!direct) {
        // the descent reads the operands' upper tiers: the missing ones of
        // all operands in one launch per tier
        static thread_local std::vector<spamm_matrix*> need;
        static thread_local std::vector<NormTable> htab;
        need.clear();
        htab.clear();
        for (int m = 0; m < count; ++m)
            for (const spamm_matrix* X : {A[m], B[m]}) {
                auto* Xm = const_cast<spamm_matrix*>(X);  // the upper tiers are a cache of the leaf norms
                if (Xm->tiers_valid || std::find(need.begin(), need.end(), Xm) != need.end()) continue;
                need.push_back(Xm);
                htab.push_back(norm_table(Xm));
            }
        if (!need.empty()) {
            NormTable* d_tab = (NormTable*)(ws + o_tab);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_tab, htab.data(), sizeof(NormTable) * need.size(), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_upper_norms_batched(need.data(), (int)need.size(), d_tab, s);
            for (auto* Xm : need) Xm->tiers_valid = e == hipSuccess;
        }
    }
    if (direct) {
        const int64_t* d_blk = (const int64_t*)(ws + o_blk);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + o_blk, hblk, sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = launch_cull_leaf_batched(d_desc, count, d_blk, hblk[count], s);
    } else {
        if (e == hipSuccess) e = launch_clear_masks(d_desc, count, s);
        if (e == hipSuccess)
            e = launch_cull_ex(d_desc, cp, nullptr, (uint64_t*)(ws + o_f0), (uint64_t*)(ws + o_f1), ctr,
                               st != nullptr, nullptr, items, s);
    }
    if (e == hipSuccess && sched == SPAMM_SCHED_LPT)
        e = launch_lpt_order(d_desc, count, total, maxc, (uint32_t*)(ws + o_cnt), (uint32_t*)(ws + o_hist),
                             (uint32_t*)(ws + o_offs), (uint32_t*)(ws + o_ord), lp.queue, s);
    if (e == hipSuccess && sched == SPAMM_SCHED_LIST)
        e = launch_tile_list(d_desc, count, total, (uint32_t*)(ws + o_ord), (unsigned*)(ws + o_q), lp.list_queue, s);
    if (e == hipSuccess) e = launch_leaf_typed(d_desc, lp, A[0]->dt == SPAMM_F64, s);
    // the results' leaf norms come from the epilogue; their upper tiers
    // follow when first read
    for (int m = 0; m < count; ++m) out[m]->tiers_valid = false;
    if (e == hipSuccess && st) {
        static thread_local DevCounters h;
        unsigned long long ne[kMaxBatch];
        e = hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(ne, nonempty_ctr(ctr), 8 * count, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        for (int m = 0; m < count && e == hipSuccess; ++m) {
            spamm_stats& o = st[m];
            std::memset(&o, 0, sizeof o);
            const spamm_matrix* Cm = out[m];
            o.n = Cm->n;
            o.leaf = b;
            o.levels = Cm->L;
            o.nb = Cm->nb;
            for (int l = 0; l <= Cm->L && l < kMaxLevels; ++l) o.survivors[l] = (int64_t)h.survivors[m][l];
            o.tasks = o.survivors[0];
            o.nonempty_tiles = (int64_t)ne[m];
            o.flops = 2.0 * b * (double)b * b * (double)o.tasks;
            o.culled_bound = h.culled_bound[m];
        }
        if (e == hipSuccess && (h.status & kDevCapacity)) r = set_error(SPAMM_ECAPACITY, "frontier capacity exceeded");
        for (int m = 0; m < count && e == hipSuccess && r == SPAMM_OK; ++m) {
            r = check_finite(A[m], s, "an operand A[m]");
            if (r == SPAMM_OK) r = check_finite(B[m], s, "an operand B[m]");
        }
    }
    if (!fixed) dev_free(owner, ws, s);
    if (e != hipSuccess) {
        release_fresh();
        return hip_error(e, fixed ? "spamm_multiply_batched_noalloc" : "spamm_multiply_batched");
    }
    if (!fixed)
        for (int m = 0; m < count; ++m) C[m] = out[m];
    return r;
}

}  // namespace
}  // namespace spamm

extern "C" {

spamm_status spamm_multiply_batched(int32_t count, const spamm_matrix* const* A, const spamm_matrix* const* B,
                                    const double* tau, spamm_leaf_prec prec, const spamm_tune* tune, void* stream,
                                    spamm_matrix** C, spamm_stats* st) {
    return spamm::multiply_batched_impl(count, A, B, tau, prec, tune, stream, C, st, false);
}

spamm_status spamm_multiply_batched_noalloc(int32_t count, const spamm_matrix* const* A,
                                            const spamm_matrix* const* B, const double* tau, spamm_leaf_prec prec,
                                            const spamm_tune* tune, void* stream, spamm_matrix* const* C) {
    if (!C) return spamm::set_error(SPAMM_EINVAL, "null argument");
    return spamm::multiply_batched_impl(count, A, B, tau, prec, tune, stream, const_cast<spamm_matrix**>(C),
                                        nullptr, true);
}

spamm_status spamm_sp2(const spamm_matrix* H, int64_t n_occ, double tau, int32_t max_iter, double idem_tol,
                       spamm_leaf_prec prec, void* stream, spamm_matrix** P, spamm_sp2_log* log) {
    return spamm_sp2_ex(H, n_occ, tau, max_iter, idem_tol, prec, 0, stream, P, log);
}

spamm_status spamm_sp2_ex(const spamm_matrix* H, int64_t n_occ, double tau, int32_t max_iter, double idem_tol,
                          spamm_leaf_prec prec, int32_t flags, void* stream, spamm_matrix** P,
                          spamm_sp2_log* log) {
    using namespace spamm;
    if (!H || !P) return set_error(SPAMM_EINVAL, "null argument");
    if (flags & ~(SPAMM_SP2_SYMMETRIC | SPAMM_SP2_DROPPING)) return set_error(SPAMM_EINVAL, "unknown SP2 flags");
    const bool symmetric = (flags & SPAMM_SP2_SYMMETRIC) != 0;
    const bool dropping = (flags & SPAMM_SP2_DROPPING) != 0;
    if (symmetric && dropping)
        return set_error(SPAMM_EUNSUPPORTED, "the dropping scheme is not combined with symmetric squarings");
    if (n_occ < 0 || n_occ > H->n) return set_error(SPAMM_EINVAL, "n_occ outside [0, n]");
    if (max_iter < 1 || max_iter > SPAMM_SP2_MAX_ITER) return set_error(SPAMM_EINVAL, "max_iter outside [1, 256]");
    if (!(idem_tol >= 0.0) || !std::isfinite(idem_tol)) return set_error(SPAMM_EINVAL, "idem_tol must be >= 0");
    spamm_status v = check_operands(H, H, tau, prec);
    if (v != SPAMM_OK) return v;
    // the dropping scheme's tau is the drop threshold; its squarings keep
    // every pair of present (non-zero) tiles
    const double tau_drop = dropping ? tau : 0.0;
    if (dropping) tau = kPresentTau;
    if (prec == SPAMM_LEAF_F64 || H->dt != SPAMM_F32)
        return set_error(SPAMM_EUNSUPPORTED, "SP2 runs on FP32 tiles with FP32 or split 16-bit leaves");
    if (H->nb * H->nb > (int64_t)UINT32_MAX) return set_error(SPAMM_EUNSUPPORTED, "SP2 needs nb^2 < 2^32 tiles");
    if (H->view) return set_error(SPAMM_EUNSUPPORTED, "SP2 takes a packed H (spamm_build), not a view");
    hipStream_t s = (hipStream_t)stream;
    (void)num_cus();  // device query outside the capture
    spamm_matrix* X[2] = {nullptr, nullptr};
    spamm_matrix* owner = nullptr;  // allocator context of the scratch block
    void* scratch = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = nullptr;
    spamm_status r = SPAMM_OK;
    const int64_t nb = H->nb;
    const size_t part_bytes = (size_t)(nb * nb + nb) * 8;
    const size_t off_part = 0, off_lo = (part_bytes + 255) & ~(size_t)255;
    const size_t off_hi = off_lo + (((size_t)H->n * 8 + 255) & ~(size_t)255);
    const size_t off_st = off_hi + (((size_t)H->n * 8 + 255) & ~(size_t)255);
    const size_t off_e = off_st + ((sizeof(Sp2State) + 255) & ~(size_t)255);
    const size_t off_list = off_e + (((size_t)(nb * nb + 1) * 8 + 255) & ~(size_t)255);
    const size_t total = off_list + (size_t)nb * nb * 4;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
        if (scratch && owner) dev_free(owner, scratch, s);
        scratch = nullptr;
        for (auto* x : X)
            if (x) release(x);
    };
    for (int i = 0; i < 2 && r == SPAMM_OK; ++i) {
        X[i] = new_handle(H->n, H->b, SPAMM_F32);
        X[i]->last_stream = s;
        r = alloc_storage(X[i], s);
        if (r == SPAMM_OK) r = ensure_scratch(X[i], s);
    }
    if (r == SPAMM_OK) {
        owner = X[0];
        scratch = dev_alloc(owner, total, s);
        if (!scratch) r = set_error(SPAMM_ENOMEM, "SP2 scratch allocation failed");
    }
    if (r != SPAMM_OK) {
        cleanup();
        return r;
    }
    char* base = (char*)scratch;
    double* part = (double*)(base + off_part);
    double* glo = (double*)(base + off_lo);
    double* ghi = (double*)(base + off_hi);
    Sp2State* st = (Sp2State*)(base + off_st);
    double* etile = (double*)(base + off_e);
    uint32_t* tile_list = (uint32_t*)(base + off_list);
    double* eout = etile + nb * nb;
    static thread_local Sp2State h;
    std::memset(&h, 0, sizeof h);
    h.n_occ = (double)n_occ;
    h.tol = idem_tol;
    h.max_iter = max_iter;
    auto fail = [&](hipError_t e, const char* what) {
        r = hip_error(e, what);
        cleanup();
        return r;
    };
    hipError_t e = hipMemcpyAsync(st, &h, sizeof h, hipMemcpyHostToDevice, s);
    if (symmetric) {
        // symmetric squarings mirror every tile below the diagonal: H must be
        // exactly symmetric (then X_0 and every X_m are)
        unsigned bad = 0;
        if (e == hipSuccess) e = launch_check_symmetric(H, &st->sym_bad, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, &st->sym_bad, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && bad) {
            cleanup();
            return set_error(SPAMM_EINVAL, "symmetric SP2 needs an exactly symmetric H");
        }
    }
    if (e == hipSuccess) e = launch_gershgorin(H, glo, ghi, st, s);
    if (e == hipSuccess) e = launch_sp2_init(H, X[0], part, st, s);
    // descriptors of the two directions X0 -> X1 and X1 -> X0
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        spamm_matrix* src = X[i];
        spamm_matrix* dst = X[1 - i];
        ProdDesc d = make_desc(src, src, dst, tau);
        d.nonempty = nullptr;  // SP2 reports no per-product tile counts
        d.sym_upper = symmetric;
        d.sp2_part = part;
        d.X = src->tiles;
        dst->ps->host_desc = d;
        dst->ps->desc_valid = false;  // differs from any plain product's descriptor
        e = hipMemcpyAsync(dst->ps->desc, &dst->ps->host_desc, sizeof d, hipMemcpyHostToDevice, s);
    }
    // product counters start at zero; each step's finalize leaves them so
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipMemsetAsync(X[i]->ps->ctr, 0, sizeof(DevCounters), s);
    // the second X buffer starts as an all-zero matrix that is known to be
    // zero (exponents -128, norms 0): a listing step writes only the tiles it
    // lists (as every later step does) instead of every tile of the fresh
    // buffer, and the tiles no step writes hold their zeros
    if (tau > 0.0 || symmetric) {
        const size_t tb = (size_t)(nb * nb) * X[1]->b * X[1]->b * X[1]->elem;
        if (e == hipSuccess) e = hipMemsetAsync(X[1]->tiles, 0, tb, s);
        if (e == hipSuccess) e = hipMemsetAsync(X[1]->norms, 0, (size_t)(nb * nb) * sizeof(double), s);
        if (e == hipSuccess) e = hipMemsetAsync(X[1]->texp, 0x80, (size_t)(nb * nb), s);
    }
    if (e != hipSuccess) return fail(e, "spamm_sp2 setup");
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return fail(e, "hipStreamCreate");
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return fail(e, "hipStreamBeginCapture");
    const int* d_branch = &st->branch;
    const int* d_active = &st->active;
    for (int m = 0; m < max_iter && r == SPAMM_OK; ++m) {
        spamm_matrix* src = X[m & 1];
        spamm_matrix* dst = X[(m + 1) & 1];
        // tau > 0: the leaf launch visits the listed tiles only; at tau = 0
        // every tile has kept products and the static full grid is faster
        // (symmetric squarings always list: tiles below the diagonal are
        // written by their mirrors, never by a block of their own)
        r = enqueue_product(src, src, dst, tau, prec, cs, 0, 1, d_branch, d_active, dst->ps->desc,
                            (tau > 0.0 || symmetric) ? tile_list : nullptr, st);
        if (r == SPAMM_OK && dropping) {
            e = launch_sp2_drop(dst, part, tau_drop * tau_drop, d_active, cs);
            if (e != hipSuccess) r = hip_error(e, "sp2 drop launch");
        }
        if (r == SPAMM_OK) {
            e = launch_sp2_finalize(part, nb, &dst->ps->ctr->survivors[0][0], st, m, cs);
            if (e != hipSuccess) r = hip_error(e, "sp2 finalize launch");
        }
    }
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (r != SPAMM_OK) {
        cleanup();
        return r;
    }
    if (ec != hipSuccess) return fail(ec, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
        return fail(e, "hipGraphInstantiate");
    if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return fail(e, "hipGraphLaunch");
    if ((e = hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e, "state copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "hipStreamSynchronize");
    const int res = h.result_step & 1;
    double energy = 0.0;
    e = launch_energy(X[res], H, etile, eout, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&energy, eout, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(e, "spamm_sp2 energy");
    if (log) {
        std::memset(log, 0, sizeof *log);
        log->iterations = h.iter;
        log->converged = h.converged;
        log->stagnated = h.stagnated;
        log->result_step = h.result_step;
        for (int m = 0; m < h.iter && m < SPAMM_SP2_MAX_ITER; ++m) {
            log->trace[m] = h.trace[m];
            log->idem[m] = h.idem[m];
            log->branch[m] = h.br[m];
            log->tasks[m] = (int64_t)h.tasks[m];
        }
        log->final_trace = h.result_step == h.iter ? h.cur_trace : h.trace[h.result_step];
        log->energy = energy;
        log->eps_min = h.eps_min;
        log->eps_max = h.eps_max;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    exec = nullptr;
    graph = nullptr;
    cs = nullptr;
    dev_free(owner, scratch, s);
    scratch = nullptr;
    // the steps after convergence were skipped on the device, so the tier
    // state recorded while capturing may not hold: form P's tiers afresh
    X[res]->tiers_valid = false;
    *P = X[res];
    X[res] = nullptr;
    cleanup();
    if (!h.converged && !h.stagnated)
        return set_error(SPAMM_ENOCONV, "SP2 met no stopping rule within max_iter steps");
    return SPAMM_OK;
}

}  // extern "C"

namespace spamm {

spamm_status multiply_count(const spamm_matrix* A, const spamm_matrix* B, double tau, spamm_leaf_prec prec,
                            hipStream_t s, spamm_matrix** C, int64_t* tasks) {
    if (!C || !tasks) return set_error(SPAMM_EINVAL, "null argument");
    spamm_status v = check_operands(A, B, tau, prec);
    if (v != SPAMM_OK) return v;
    const spamm_dtype cdt = prec == SPAMM_LEAF_F64 ? SPAMM_F64 : SPAMM_F32;
    spamm_matrix* Cm = *C;
    if (Cm && (Cm == A || Cm == B || Cm->view || Cm->n != A->n || Cm->b != A->b || Cm->dt != cdt))
        return set_error(SPAMM_EINVAL, "C does not fit the product");
    bool fresh = false;
    if (!Cm) {
        Cm = new_handle(A->n, A->b, cdt);
        fresh = true;
        spamm_status r = alloc_storage(Cm, s);
        if (r != SPAMM_OK) {
            release(Cm);
            return r;
        }
    }
    Cm->last_stream = s;
    spamm_status r = ensure_scratch(Cm, s);
    if (r == SPAMM_OK)
        r = enqueue_product(A, B, Cm, tau, prec, s, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, true);
    if (r != SPAMM_OK) {
        if (fresh) release(Cm);
        return r;
    }
    *C = Cm;
    spamm_stats st;
    r = read_stats(Cm, s, &st, tau);
    *tasks = st.tasks;
    return r;
}

}  // namespace spamm
