// Product-space cull of the SpAMM recursion (section 2, Eq. 4; the octree of
// Figure 1) as level-synchronous passes on gfx950.
//
// The frontier of tier l holds the kept octree nodes (m, I, J, K) of every
// product in the batch.  One launch per tier expands each node into its 8
// children and keeps a child iff !(S_A[l-1][I',K'] * S_B[l-1][K',J'] < tau^2)
// (with the depth-scaled schedule of section 2, tau / 8^k at depth k below
// the root: tau^2 scaled by 2^-6k, exact in FP64);
// survivors are compacted with a block-wide exclusive prefix scan and one
// atomic reservation per block.  Children at the leaf tier are not
// compacted: they set bit K of the C tile (I, J) in a bitmask, which gives
// every C tile its kept K in ascending order with no sort.
//
// Roots enter as virtual items: at tier l the products whose quadtree has l
// tiers test their root and expand it in the same launch, so a batch of
// unequal sizes is culled with one launch per tier.
#include "spamm_internal.hpp"

namespace spamm {
namespace {

constexpr int kCullThreads = 256;
constexpr int kTopThreads = 1024;  // the single-block launch of the small upper tiers

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int d = kWave / 2; d >= 1; d /= 2) v += __shfl_xor(v, d, kWave);
    return v;
}

// One pass over the items of tier l (the stored frontier, then the virtual
// roots).  ONE_BLOCK: the whole tier is handled by this block, which keeps the
// frontier sizes in LDS (s_count) instead of the global counters, so several
// small tiers run in one launch.
template <bool ONE_BLOCK, int NT>
__device__ void cull_pass(const ProdDesc* __restrict__ desc, int nprod, int l, const uint64_t* __restrict__ in,
                          uint64_t* __restrict__ out, DevCounters* __restrict__ ctr, int64_t out_cap, int want_bound,
                          unsigned* wave_tot, unsigned long long* block_base, unsigned long long* s_count,
                          unsigned long long* s_surv) {
    const int64_t P = ONE_BLOCK ? (int64_t)s_count[l] : (int64_t)ctr->front_count[l];
    const int64_t items = P + nprod;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int c = l - 1;  // child tier
    const int64_t first = ONE_BLOCK ? 0 : (int64_t)blockIdx.x * NT;
    const int64_t stride = ONE_BLOCK ? NT : (int64_t)gridDim.x * NT;

    for (int64_t base = first; base < items; base += stride) {
        const int64_t idx = base + threadIdx.x;
        uint32_t m = 0, I = 0, J = 0, K = 0;
        bool have = false;
        if (idx < P) {
            const uint64_t key = in[idx];
            m = key_m(key);
            I = key_i(key);
            J = key_j(key);
            K = key_k(key);
            have = true;
        } else if (idx < items) {
            m = (uint32_t)(idx - P);
            const ProdDesc& d = desc[m];
            if (d.L == l || (l == 1 && d.L == 0)) {
                // root of product m: Eq. (4) tests it like any other node
                const double sa = d.SA[d.lvl_off[d.L]], sb = d.SB[d.lvl_off[d.L]];
                if (!(sa * sb < d.tau2)) {
                    atomicAdd(&ctr->survivors[m][d.L], 1ull);
                    if (d.L == 0) {
                        atomicOr((unsigned long long*)&d.mask[0], 1ull);
                    } else {
                        have = true;
                    }
                } else if (want_bound) {
                    atomicAdd(&ctr->culled_bound[m], sqrt(sa) * sqrt(sb));
                }
            }
        }
        unsigned keep = 0;  // bit q set: child q kept (q = i2*4 + j2*2 + k2)
        unsigned long long leaf_kept = 0;
        double bound = 0.0;
        if (have) {
            const ProdDesc& d = desc[m];
            const int mc = d.lvl_m[c];
            const double* SA = d.SA + d.lvl_off[c];
            const double* SB = d.SB + d.lvl_off[c];
            // tau^2 of the children's depth L - c (the root, depth 0, uses tau^2)
            const double t2 = d.depth_tau ? ldexp(d.tau2, -6 * (d.L - c)) : d.tau2;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t Ic = 2 * I + (q >> 2), Jc = 2 * J + ((q >> 1) & 1), Kc = 2 * K + (q & 1);
                if ((int)Ic >= mc || (int)Jc >= mc || (int)Kc >= mc) continue;
                // symmetric squaring: a node with I > J holds only tiles below
                // the diagonal, which are mirrored, not formed
                if (d.sym_upper && Ic > Jc) continue;
                const double sa = SA[(int64_t)Ic * mc + Kc];
                const double sb = SB[(int64_t)Kc * mc + Jc];
                if (sa * sb < t2) {
                    if (want_bound) bound += sqrt(sa) * sqrt(sb);
                    continue;
                }
                if (c == 0) {
                    uint64_t* w = d.mask + ((int64_t)Ic * mc + Jc) * d.W + (Kc >> 6);
                    atomicOr((unsigned long long*)w, 1ull << (Kc & 63));
                    ++leaf_kept;
                } else {
                    keep |= 1u << q;
                }
            }
        }
        // survivors of this tier per product: one atomic per uniform wave
        const unsigned nk = __popc(keep);
        {
            const unsigned long long mine = (unsigned long long)nk + leaf_kept;
            const uint32_t m0 = __shfl(m, 0, kWave);
            const bool uniform = __all(!(have) || m == m0);
            if (uniform) {
                const unsigned long long s = wave_sum_u64(mine);
                // one product per launch: the block adds its waves in LDS and
                // its caller adds the block total once
                if (lane == 0 && s) {
                    if (s_surv) atomicAdd(s_surv, s);
                    else atomicAdd(&ctr->survivors[m0][c], s);
                }
            } else if (mine) {
                atomicAdd(&ctr->survivors[m][c], mine);
            }
            // the culled-node bound: one atomic per wave of one product
            // (per thread, the adds to one address serialise)
            if (want_bound) {
                if (uniform) {
                    double sb = bound;
                    for (int d = kWave / 2; d >= 1; d /= 2) sb += __shfl_xor(sb, d, kWave);
                    if (lane == 0 && sb > 0.0) atomicAdd(&ctr->culled_bound[m0], sb);
                } else if (bound > 0.0) {
                    atomicAdd(&ctr->culled_bound[m], bound);
                }
            }
        }
        if (c == 0) continue;  // leaf tier: nothing to compact
        // block-wide exclusive scan of the per-thread child counts
        unsigned incl = nk;
        for (int d = 1; d < kWave; d *= 2) {
            const unsigned o = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += o;
        }
        if (lane == kWave - 1) wave_tot[wid] = incl;
        __syncthreads();
        unsigned wave_off = 0, block_tot = 0;
        for (int w = 0; w < NT / kWave; ++w) {
            if (w < wid) wave_off += wave_tot[w];
            block_tot += wave_tot[w];
        }
        if (threadIdx.x == 0) {
            if (ONE_BLOCK) {
                *block_base = s_count[c];
                s_count[c] += block_tot;
            } else {
                *block_base = block_tot ? atomicAdd(&ctr->front_count[c], (unsigned long long)block_tot) : 0ull;
            }
        }
        __syncthreads();
        int64_t pos = (int64_t)*block_base + wave_off + (incl - nk);
        if (keep) {
            if (pos + nk > out_cap) {
                atomicOr(&ctr->status, kDevCapacity);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (keep & (1u << q))
                        out[pos++] = node_key(m, 2 * I + (q >> 2), 2 * J + ((q >> 1) & 1), 2 * K + (q & 1));
            }
        }
        __syncthreads();
    }
}


__global__ void __launch_bounds__(kCullThreads)
    k_cull_tier(const ProdDesc* __restrict__ desc, int nprod, int l, const uint64_t* __restrict__ in,
                uint64_t* __restrict__ out, DevCounters* __restrict__ ctr, int64_t out_cap, int want_bound,
                const int* __restrict__ active) {
    if (active && *active == 0) return;
    __shared__ unsigned wave_tot[kCullThreads / kWave];
    __shared__ unsigned long long block_base;
    __shared__ unsigned long long s_surv;
    if (threadIdx.x == 0) s_surv = 0;
    __syncthreads();
    cull_pass<false, kCullThreads>(desc, nprod, l, in, out, ctr, out_cap, want_bound, wave_tot, &block_base,
                                   nullptr, nprod == 1 ? &s_surv : nullptr);
    __syncthreads();
    if (threadIdx.x == 0 && s_surv) atomicAdd(&ctr->survivors[0][l - 1], s_surv);
}

// Tiers top .. stop + 1 in one block (small frontiers): the frontier of tier l
// lives in buffer (l & 1) as in the per-tier launches, and the sizes reach the
// global counters for the launches that follow.
__global__ void __launch_bounds__(kTopThreads)
    k_cull_top(const ProdDesc* __restrict__ desc, int nprod, int top, int stop, uint64_t* __restrict__ front0,
               uint64_t* __restrict__ front1, DevCounters* __restrict__ ctr, int64_t out_cap, int want_bound,
               const int* __restrict__ active) {
    if (active && *active == 0) return;
    __shared__ unsigned wave_tot[kTopThreads / kWave];
    __shared__ unsigned long long block_base;
    __shared__ unsigned long long s_count[kMaxLevels];
    if (threadIdx.x < kMaxLevels) s_count[threadIdx.x] = 0;
    __syncthreads();
    for (int l = top; l > stop; --l) {
        const uint64_t* in = (l & 1) ? front1 : front0;
        uint64_t* out = ((l - 1) & 1) ? front1 : front0;
        cull_pass<true, kTopThreads>(desc, nprod, l, in, out, ctr, out_cap, want_bound, wave_tot, &block_base,
                                     s_count, nullptr);
        __syncthreads();  // this tier's stores are read by the next pass of the same block
    }
    if (threadIdx.x < kMaxLevels) ctr->front_count[threadIdx.x] = s_count[threadIdx.x];
}

// The frontier of tier s of a single product straight from the flat rule:
// node (I,J,K) passes iff !(S_A[s][I,K] * S_B[s][K,J] < tau^2).  Tier norms
// are FP64 sums of their children's non-negative norms (rounding is
// monotone), so every ancestor of a passing node passes too and the descent
// from the root keeps exactly this set; only the depth-scaled schedule, whose
// thresholds differ per tier, needs the descent.  Each block takes a
// contiguous range of nodes in two passes (count, then store), so the
// frontier counter sees one atomic per block.  (This path runs without
// statistics; the survivors of tier s are not counted.)
__device__ inline bool enum_keep(const ProdDesc& d, const double* SA, const double* SB, int ms, int64_t idx,
                                 uint32_t& I, uint32_t& J, uint32_t& K) {
    I = (uint32_t)(idx / ((int64_t)ms * ms));
    J = (uint32_t)((idx / ms) % ms);
    K = (uint32_t)(idx % ms);
    return !(SA[(int64_t)I * ms + K] * SB[(int64_t)K * ms + J] < d.tau2) && !(d.sym_upper && I > J);
}

__global__ void __launch_bounds__(kCullThreads)
    k_cull_enum(const ProdDesc* __restrict__ desc, int s, int ms, uint64_t* __restrict__ out,
                DevCounters* __restrict__ ctr, int64_t out_cap, const int* __restrict__ active) {
    if (active && *active == 0) return;
    __shared__ unsigned wave_tot[kCullThreads / kWave];
    __shared__ unsigned long long block_base;
    const ProdDesc& d = desc[0];
    const double* SA = d.SA + d.lvl_off[s];
    const double* SB = d.SB + d.lvl_off[s];
    const int64_t total = (int64_t)ms * ms * ms;
    const int64_t per = ((total + gridDim.x - 1) / gridDim.x + kCullThreads - 1) / kCullThreads * kCullThreads;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < total ? lo + per : total;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t I, J, K;
    // pass 1: this block's count
    unsigned cnt = 0;
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += kCullThreads) cnt += enum_keep(d, SA, SB, ms, idx, I, J, K);
    for (int dd = kWave / 2; dd >= 1; dd /= 2) cnt += __shfl_xor(cnt, dd, kWave);
    if (lane == 0) wave_tot[wid] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int w = 0; w < kCullThreads / kWave; ++w) tot += wave_tot[w];
        block_base = tot ? atomicAdd(&ctr->front_count[s], (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    // pass 2: stores in node order within the block
    unsigned long long run = block_base;
    for (int64_t base = lo; base < hi; base += kCullThreads) {
        const int64_t idx = base + threadIdx.x;
        const bool keep = idx < hi && enum_keep(d, SA, SB, ms, idx, I, J, K);
        const unsigned long long bal = __ballot(keep);
        __syncthreads();  // wave_tot of the previous chunk has been read
        if (lane == 0) wave_tot[wid] = (unsigned)__popcll(bal);
        __syncthreads();
        unsigned wave_off = 0, chunk_tot = 0;
        for (int w = 0; w < kCullThreads / kWave; ++w) {
            if (w < wid) wave_off += wave_tot[w];
            chunk_tot += wave_tot[w];
        }
        if (keep) {
            const int64_t pos = (int64_t)run + wave_off + __popcll(bal & ((1ull << lane) - 1ull));
            if (pos >= out_cap) atomicOr(&ctr->status, kDevCapacity);
            else out[pos] = node_key(0, I, J, K);
        }
        run += chunk_tot;
    }
}

// The leaf tier of a single product straight from the flat rule, without
// the tiers above (every ancestor of a passing triple passes, see
// enum_keep): bit K of C tile (I, J) is set iff
// !(S_A[I,K] * S_B[K,J] < tau^2).  Block (I, y) forms every mask word of
// the tiles (I, 64y + j) with up to four words at a time: wave (v, q) of
// the block takes quarter q (16 K) of word v of the group, lane j testing
// tile (I, 64y + j) and reading row K of S_B coalesced across the lanes
// (S_A[I,K] is one value per wave).  The quarters are OR-ed in LDS and each
// word is stored once, so every mask word is written (no clearing, no
// atomics per triple) and the kept K of a tile stay in ascending order.
//
// SP2 (list != NULL): with all of a tile's words at hand the block also
// decides whether the step writes the tile (kept products, or X_m or the
// previous result nonzero there; for symmetric squarings tiles below the
// diagonal are written by their mirrors), gives the others zero SP2
// partials and appends the rest to the step's tile list.
constexpr int kLeafQuarters = 4;
constexpr int kLeafWords = 4;  // words per group (block of kLeafWords x kLeafQuarters waves)
__global__ void __launch_bounds__(kLeafWords * kLeafQuarters * kWave)
    k_cull_leaf(const ProdDesc* __restrict__ desc, DevCounters* __restrict__ ctr, uint32_t* __restrict__ list,
                Sp2State* __restrict__ st, const int* __restrict__ active) {
    if (active && *active == 0) return;
    const ProdDesc& d = desc[0];
    const int nb = d.nb, W = d.W;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int q = wid % kLeafQuarters, v = wid / kLeafQuarters;
    const int group = (int)(blockDim.x / (kLeafQuarters * kWave));  // words per group: min(W, kLeafWords)
    const int I = blockIdx.x, J = blockIdx.y * kWave + lane;
    constexpr int KQ = 64 / kLeafQuarters;
    const bool live = J < nb && !(d.sym_upper && I > J);
    const double t2 = d.tau2;
    __shared__ unsigned long long s_bits[kLeafWords * kLeafQuarters][kWave];
    __shared__ unsigned long long s_any[kLeafWords][kWave], s_kept[kLeafWords][kWave];
    unsigned long long kept = 0, any = 0;  // (waves q == 0: over their words)
    for (int w0 = 0; w0 < W; w0 += group) {
        const int w = w0 + v;
        const int k0 = w * 64 + q * KQ, kn = min(KQ, nb - k0);  // kn <= 0: quarter past the last K
        unsigned long long bits = 0;
        if (live && w < W && kn > 0) {
            const double* SA = d.SA + d.lvl_off[0] + (int64_t)I * nb + k0;
            const double* SB = d.SB + d.lvl_off[0] + (int64_t)k0 * nb + J;
#pragma unroll 8
            for (int k = 0; k < kn; ++k) bits |= (unsigned long long)!(SA[k] * SB[(int64_t)k * nb] < t2) << k;
            bits <<= q * KQ;
        }
        s_bits[wid][lane] = bits;
        __syncthreads();
        if (q == 0 && w < W) {
            for (int r = 1; r < kLeafQuarters; ++r) bits |= s_bits[wid + r][lane];
            if (J < nb) d.mask[((int64_t)I * nb + J) * W + w] = bits;
            kept += (unsigned long long)__popcll(bits);
            any |= bits;
        }
        __syncthreads();
    }
    if (q == 0) {
        s_any[v][lane] = any;
        s_kept[v][lane] = kept;
    }
    __syncthreads();
    if (wid != 0) return;
    for (int r = 1; r < group; ++r) {
        any |= s_any[r][lane];
        kept += s_kept[r][lane];
    }
    // kept triples (the product's task count, when someone reads it): one
    // atomic per block
    if (ctr) {
        const unsigned long long c = wave_sum_u64(kept);
        if (lane == 0 && c) atomicAdd(&ctr->survivors[0][0], c);
    }
    if (!list) return;
    const int64_t tiles = (int64_t)nb * nb, t = (int64_t)I * nb + J;
    bool need = false;
    if (live) {
        const int64_t mirror = (int64_t)J * nb + I;
        need = any != 0 || d.SA[t] != 0.0 || d.eC[t] != -128 || (d.sym_upper && I < J && d.eC[mirror] != -128);
        if (!need) {
            d.sp2_part[t] = 0.0;
            if (I == J) d.sp2_part[tiles + I] = 0.0;
            if (d.sym_upper && I < J) d.sp2_part[mirror] = 0.0;
        }
    }
    const unsigned long long m = __ballot(need);
    if (m == 0) return;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(&st->list_count, (unsigned)__popcll(m));
    base = (unsigned)__shfl((int)base, 0, kWave);
    if (need) list[base + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)t;
}

// The direct leaf pass for a batch of flat-threshold products without
// statistics: as k_cull_leaf, one block per (product, tile row I, 64 tiles
// J), the four waves taking the quarters of each mask word in turn.
// blk_off[m] is the first block of product m (ascending); the kept counts
// are not formed (nothing reads them without statistics).
__global__ void __launch_bounds__(kLeafQuarters * kWave)
    k_cull_leaf_batched(const ProdDesc* __restrict__ desc, int nprod, const int64_t* __restrict__ blk_off) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nprod - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk_off[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const ProdDesc& d = desc[lo];
    const int nb = d.nb, W = d.W, ny = (nb + kWave - 1) / kWave;
    const int64_t local = b - blk_off[lo];
    const int I = (int)(local / ny);
    const int lane = threadIdx.x & (kWave - 1);
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int J = (int)(local % ny) * kWave + lane;
    constexpr int KQ = 64 / kLeafQuarters;
    const bool live = J < nb;
    const double t2 = d.tau2;
    __shared__ unsigned long long s_bits[kLeafQuarters][kWave];
    for (int w = 0; w < W; ++w) {
        const int k0 = w * 64 + q * KQ, kn = min(KQ, nb - k0);
        unsigned long long bits = 0;
        if (live && kn > 0) {
            const double* SA = d.SA + d.lvl_off[0] + (int64_t)I * nb + k0;
            const double* SB = d.SB + d.lvl_off[0] + (int64_t)k0 * nb + J;
#pragma unroll 8
            for (int k = 0; k < kn; ++k) bits |= (unsigned long long)!(SA[k] * SB[(int64_t)k * nb] < t2) << k;
            bits <<= q * KQ;
        }
        s_bits[q][lane] = bits;
        __syncthreads();
        if (q == 0 && live) {
            for (int r = 1; r < kLeafQuarters; ++r) bits |= s_bits[r][lane];
            d.mask[((int64_t)I * nb + J) * W + w] = bits;
        }
        __syncthreads();
    }
}

// Counters, per-product non-empty tile counts and (single product) the leaf
// bitmask, zeroed in one launch.
__global__ void k_cull_prep(DevCounters* ctr, unsigned long long* nonempty, int nprod, uint64_t* mask,
                            int64_t words, const int* active) {
    if (active && *active == 0) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    if (t < kMaxLevels) ctr->front_count[t] = 0;
    if (t == 0) ctr->status = 0;
    for (int64_t i = t; i < (int64_t)nprod * kMaxLevels; i += nt) ctr->survivors[i / kMaxLevels][i % kMaxLevels] = 0;
    for (int64_t i = t; i < nprod; i += nt) {
        ctr->culled_bound[i] = 0.0;
        if (nonempty) nonempty[i] = 0;
    }
    for (int64_t i = t; i < words; i += nt) mask[i] = 0;
}

// Batch: block (m, y) clears slice y of product m's leaf bitmask.
__global__ void k_clear_masks(const ProdDesc* __restrict__ desc) {
    const ProdDesc& d = desc[blockIdx.x];
    const int64_t words = (int64_t)d.nb * d.nb * d.W;
    const int64_t per = (words + gridDim.y - 1) / gridDim.y;
    const int64_t lo = per * blockIdx.y, hi = lo + per < words ? lo + per : words;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) d.mask[i] = 0;
}

__global__ void k_task_keys(const ProdDesc* __restrict__ desc, int64_t nb, int W, const uint64_t* __restrict__ mask,
                            uint64_t* __restrict__ out, unsigned long long* count, int64_t cap) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * nb) return;
    const int64_t I = t / nb, J = t % nb;
    for (int w = 0; w < W; ++w) {
        uint64_t bits = mask[t * W + w];
        while (bits) {
            const int k = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            const unsigned long long p = atomicAdd(count, 1ull);
            if ((int64_t)p < cap) out[p] = ((uint64_t)I << 42) | ((uint64_t)J << 21) | (uint64_t)(w * 64 + k);
        }
    }
}

}  // namespace

// Tier-by-tier cull; `plan.front_cap` bounds each frontier buffer.
hipError_t launch_cull_ex(const ProdDesc* d_desc, const CullPlan& plan, uint64_t* mask, uint64_t* front0,
                          uint64_t* front1, DevCounters* ctr, int want_bound, const int* active,
                          const int64_t* tier_items, hipStream_t s) {
    if (!plan.skip_prep) {
        // (a batch clears its masks with launch_clear_masks; the direct leaf
        // pass writes every word)
        const int64_t words = mask && !plan.leaf_direct ? plan.mask_words : 0;
        int64_t blocks = (words + 255) / 256;
        blocks = blocks < 8 ? 8 : (blocks > 2048 ? 2048 : blocks);
        hipLaunchKernelGGL(k_cull_prep, dim3((unsigned)blocks), dim3(256), 0, s, ctr, plan.nonempty, plan.count, mask,
                           words, active);
    }
    const int top = plan.Lmax < 1 ? 1 : plan.Lmax;
    int l = top;
    if (plan.leaf_direct) {
        const unsigned nb = (unsigned)plan.leaf_nb;
        const unsigned W = (nb + 63) / 64, group = W < (unsigned)kLeafWords ? W : (unsigned)kLeafWords;
        hipLaunchKernelGGL(k_cull_leaf, dim3(nb, (nb + kWave - 1) / kWave), dim3(group * kLeafQuarters * kWave), 0, s,
                           d_desc, plan.uncounted ? nullptr : ctr, plan.sp2_list, plan.sp2_state, active);
        return hipGetLastError();
    }
    if (plan.flat_start >= 1) {
        // tier flat_start enumerated directly; its frontier lives in buffer (flat_start & 1)
        const int fs = plan.flat_start;
        const int64_t cells = (int64_t)plan.flat_m * plan.flat_m * plan.flat_m;
        int64_t blocks = (cells + kCullThreads - 1) / kCullThreads;
        const int64_t maxb = (int64_t)num_cus();  // one block per CU: few counter atomics
        blocks = blocks < 1 ? 1 : (blocks > maxb ? maxb : blocks);
        hipLaunchKernelGGL(k_cull_enum, dim3((unsigned)blocks), dim3(kCullThreads), 0, s, d_desc, fs, plan.flat_m,
                           (fs & 1) ? front1 : front0, ctr, plan.front_cap, active);
        l = fs;
    } else {
        // tiers whose items fit a few passes of one block go to one launch
        constexpr int64_t kOneBlockItems = 4 * kTopThreads;
        int stop = top;
        while (stop >= 1 && tier_items[stop] + plan.count <= kOneBlockItems) --stop;
        if (stop < top) {
            hipLaunchKernelGGL(k_cull_top, dim3(1), dim3(kTopThreads), 0, s, d_desc, plan.count, top, stop, front0,
                               front1, ctr, plan.front_cap, want_bound, active);
            l = stop;
        }
    }
    for (; l >= 1; --l) {
        // frontier of tier l lives in buffer (l & 1); children go to ((l-1) & 1)
        const uint64_t* in = (l & 1) ? front1 : front0;
        uint64_t* out = ((l - 1) & 1) ? front1 : front0;
        int64_t items = tier_items[l] + plan.count;
        int64_t blocks = (items + kCullThreads - 1) / kCullThreads;
        const int64_t maxb = (int64_t)num_cus() * 8;
        blocks = blocks < 1 ? 1 : (blocks > maxb ? maxb : blocks);
        hipLaunchKernelGGL(k_cull_tier, dim3((unsigned)blocks), dim3(kCullThreads), 0, s, d_desc, plan.count, l,
                           in, out, ctr, plan.front_cap, want_bound, active);
    }
    return hipGetLastError();
}

hipError_t launch_cull_leaf_batched(const ProdDesc* d_desc, int nprod, const int64_t* d_blk_off, int64_t blocks,
                                   hipStream_t s) {
    if (blocks > 0)
        hipLaunchKernelGGL(k_cull_leaf_batched, dim3((unsigned)blocks), dim3(kLeafQuarters * kWave), 0, s, d_desc, nprod,
                           d_blk_off);
    return hipGetLastError();
}

hipError_t launch_clear_masks(const ProdDesc* d_desc, int nprod, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_masks, dim3((unsigned)nprod, 64), dim3(256), 0, s, d_desc);
    return hipGetLastError();
}

hipError_t launch_task_keys(const ProdDesc* d_desc, int64_t nb, int W, const uint64_t* mask, uint64_t* keys_out,
                            unsigned long long* count, int64_t cap, hipStream_t s) {
    const int64_t tiles = nb * nb;
    hipLaunchKernelGGL(k_task_keys, dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, s, d_desc, nb, W, mask,
                       keys_out, count, cap);
    return hipGetLastError();
}

}  // namespace spamm
