// Leaf-product schedule for the persistent launch: every C tile's work is its
// number of kept K (a popcount of its leaf bitmask); tiles are ordered
// largest first (LPT) by a counting sort on that number, so a batch of
// products of very different sizes drains evenly over the resident blocks.
#include "spamm_internal.hpp"

namespace spamm {
namespace {

__device__ inline int product_of(const ProdDesc* desc, int nprod, int64_t t) {
    int lo = 0, hi = nprod - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Kept-K count of global C tile t (0 past the end).
__device__ inline uint32_t tile_count(const ProdDesc* desc, int nprod, int64_t total, int64_t t) {
    if (t >= total) return 0;
    const ProdDesc& d = desc[product_of(desc, nprod, t)];
    const uint64_t* w = d.mask + (t - d.tile_base) * d.W;
    uint32_t c = 0;
    for (int i = 0; i < d.W; ++i) c += (uint32_t)__popcll(w[i]);
    return c;
}

// Empty tiles (count 0) are usually the majority: each wave adds them to
// hist[0] with one atomic instead of one per tile.
__global__ void k_tile_counts(const ProdDesc* __restrict__ desc, int nprod, int64_t total, uint32_t* __restrict__ counts,
                              uint32_t* __restrict__ hist) {
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = base + threadIdx.x;
        const uint32_t c = tile_count(desc, nprod, total, t);
        if (t < total) counts[t] = c;
        const unsigned long long zero = __ballot(t < total && c == 0);
        if (lane == 0 && zero) atomicAdd(&hist[0], (unsigned)__popcll(zero));
        if (t < total && c > 0) atomicAdd(&hist[c], 1u);
    }
}

// offs[c] = number of tiles with more than c kept K (descending exclusive scan).
__global__ void __launch_bounds__(1024) k_hist_scan_desc(const uint32_t* hist, int maxc, uint32_t* offs) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (maxc + 1 + 1023) / 1024;
    // thread t owns counts [t*per, (t+1)*per) walked from the top
    uint32_t s = 0;
    for (int c = (t + 1) * per - 1; c >= t * per; --c)
        if (c <= maxc) s += hist[c];
    part[t] = s;
    __syncthreads();
    if (t == 0) {  // suffix sums over the 1024 chunks
        uint32_t run = 0;
        for (int i = 1023; i >= 0; --i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t run = part[t];
    for (int c = (t + 1) * per - 1; c >= t * per; --c) {
        if (c > maxc) continue;
        offs[c] = run;
        run += hist[c];
    }
}

// Positions in the LPT order; a wave reserves the slots of its empty tiles
// with one atomic (the order among equal counts is arbitrary either way).
__global__ void k_scatter_order(const uint32_t* __restrict__ counts, int64_t total, uint32_t* __restrict__ offs,
                                uint32_t* __restrict__ order) {
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = base + threadIdx.x;
        const uint32_t c = t < total ? counts[t] : 1u;
        const unsigned long long zero = __ballot(t < total && c == 0);
        unsigned zbase = 0;
        if (lane == 0 && zero) zbase = atomicAdd(&offs[0], (unsigned)__popcll(zero));
        zbase = (unsigned)__shfl((int)zbase, 0, 64);
        if (t >= total) continue;
        const uint32_t pos = c == 0 ? zbase + (unsigned)__popcll(zero & ((1ull << lane) - 1ull)) : atomicAdd(&offs[c], 1u);
        order[pos] = (uint32_t)t;
    }
}

// The C tiles of a product launch that need a write: a kept product, or
// stored values not known to be zero (exponent -128 marks an all-zero tile,
// whose norm is zero too).  The list order depends on the atomics; each
// tile's result does not.
// The C tiles of a batch that need a write (a kept product, or stored
// values not known to be zero), listed for the persistent leaf launch.  The
// products' first global tiles sit in LDS for the per-lane search, and each
// block reserves its part of the list with one atomic; the list order
// depends on the atomics, each tile's result does not.
__global__ void __launch_bounds__(256) k_tile_list(const ProdDesc* __restrict__ desc, int nprod, int64_t total,
                                                   uint32_t* __restrict__ list, unsigned* __restrict__ count) {
    __shared__ int64_t s_base[kMaxBatch];
    __shared__ unsigned s_wave[4];
    __shared__ unsigned s_block;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < nprod; i += blockDim.x) s_base[i] = desc[i].tile_base;
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = base + threadIdx.x;
        bool need = false;
        if (t < total) {
            int lo = 0, hi = nprod - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_base[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const ProdDesc& d = desc[lo];
            const int64_t local = t - s_base[lo];
            uint64_t any = 0;
            for (int i = 0; i < d.W; ++i) any |= d.mask[local * d.W + i];
            need = any != 0 || d.eC[local] != -128;
        }
        const unsigned long long m = __ballot(need);
        if (lane == 0) s_wave[wid] = (unsigned)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned tot = (s_wave[0] + s_wave[1]) + (s_wave[2] + s_wave[3]);
            s_block = tot ? atomicAdd(count, tot) : 0u;
        }
        __syncthreads();
        unsigned off = s_block;
        for (int w = 0; w < wid; ++w) off += s_wave[w];
        if (need) list[off + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)t;
        __syncthreads();  // s_wave and s_block are rewritten by the next chunk
    }
}

__global__ void k_zero_u32(uint32_t* p, int64_t count, unsigned long long* queue) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && queue) *queue = 0ull;
}

__global__ void k_zero_one(unsigned* p, unsigned* q) {
    *p = 0u;
    if (q) *q = 0u;
}

}  // namespace

// list: total entries; count (and the leaf launch's queue, if any) is zeroed
// first (a kernel, so the sequence can be captured in a graph).
hipError_t launch_tile_list(const ProdDesc* d_desc, int nprod, int64_t total, uint32_t* list, unsigned* count,
                            unsigned* queue, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_one, dim3(1), dim3(1), 0, s, count, queue);
    int64_t blocks = (total + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(k_tile_list, dim3((unsigned)blocks), dim3(256), 0, s, d_desc, nprod, total, list, count);
    return hipGetLastError();
}

// counts/order: total entries; hist/offs: maxc + 1 entries each; queue zeroed.
hipError_t launch_lpt_order(const ProdDesc* d_desc, int nprod, int64_t total, int maxc, uint32_t* counts,
                            uint32_t* hist, uint32_t* offs, uint32_t* order, unsigned long long* queue,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, hist, (int64_t)maxc + 1, queue);
    int64_t blocks = (total + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(k_tile_counts, dim3((unsigned)blocks), dim3(256), 0, s, d_desc, nprod, total, counts, hist);
    hipLaunchKernelGGL(k_hist_scan_desc, dim3(1), dim3(1024), 0, s, hist, maxc, offs);
    hipLaunchKernelGGL(k_scatter_order, dim3((unsigned)blocks), dim3(256), 0, s, counts, total, offs, order);
    return hipGetLastError();
}

}  // namespace spamm
