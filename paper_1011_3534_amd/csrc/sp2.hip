// TC2 / SP2 density-matrix purification on gfx950 (section 3 of the paper;
// the iteration of Niklasson, Phys. Rev. B 66, 155115, 2002).
//
// Device-side pieces: Gershgorin bounds of H, the initial X_0, tile norms of
// X_0, the per-step finalize (FP64 reductions of the epilogue partials, the
// branch for the next step and the stopping rules) and E = tr(P H).  Every
// decision stays on the device so that all steps fit one static hipGraph;
// steps after the stop see active == 0 and return at once.
#include "spamm_internal.hpp"

namespace spamm {
namespace {

constexpr double kStagBelow = 0.1;

// Fixed-order FP64 sum of x[0..count) by one block of 1024 threads: thread t
// adds x[t], x[t + 1024], ... (coalesced), then a pairwise tree.
__device__ double block_sum_fixed(const double* x, int64_t count, double* red) {
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < count; i += blockDim.x) s += x[i];
    red[t] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
        if (t < h) red[t] = red[t] + red[t + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// One wave per row i: d_i = h_ii, r_i = sum_{j != i} |h_ij|  ->  lo = d - r, hi = d + r.
// Tiles of the row's tile row with squared norm 0 hold only zeros and are not
// read: the wave tests 64 tile norms at a time and visits the others.
__global__ void __launch_bounds__(256) k_gersh_rows(const float* __restrict__ H, const double* __restrict__ S,
                                                    int64_t n, int b, int64_t nb, double* __restrict__ lo,
                                                    double* __restrict__ hi) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int64_t I = i / b, r = i % b;
    double acc = 0.0, d = 0.0;
    for (int64_t base = 0; base < nb; base += 64) {
        const int64_t kc = base + lane;
        unsigned long long m = __ballot(kc < nb && S[I * nb + kc] != 0.0);
        while (m) {
            const int64_t K = base + __builtin_ctzll(m);
            m &= m - 1;
            const float* row = H + ((I * nb + K) * b + r) * b;
            for (int c = lane; c < b; c += 64) {
                const double v = (double)row[c];
                if (K * b + c == i) d = v;
                else acc += fabs(v);
            }
        }
    }
    for (int h = 32; h >= 1; h >>= 1) {
        acc += __shfl_down(acc, h, 64);
        d += __shfl_down(d, h, 64);
    }
    if (lane == 0) {
        lo[i] = d - acc;
        hi[i] = d + acc;
    }
}

__global__ void __launch_bounds__(1024) k_gersh_reduce(const double* lo, const double* hi, int64_t n, Sp2State* st) {
    __shared__ double smin[1024], smax[1024];
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        mn = fmin(mn, lo[i]);
        mx = fmax(mx, hi[i]);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int h = blockDim.x / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + h]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->eps_min = smin[0];
        st->eps_max = smax[0];
    }
}

// X_0 = (eps_max I - H) / (eps_max - eps_min) over the padded tile storage
// (padding stays zero), one block per tile.  An off-diagonal tile of H with
// squared norm 0 is all zero, so its X_0 tile is written as zeros without
// reading H.
template <int B>
__global__ void __launch_bounds__(256) k_sp2_init_x(const float* __restrict__ H, const double* __restrict__ SH,
                                                    float* __restrict__ X, int64_t n, int64_t nb,
                                                    const Sp2State* st) {
    const int64_t tile = blockIdx.x;
    const int64_t I = tile / nb, K = tile % nb;
    constexpr int64_t TS = (int64_t)B * B;
    float* x = X + tile * TS;
    if (I != K && SH[tile] == 0.0) {
        for (int e = threadIdx.x * 4; e < B * B; e += 256 * 4)
            *reinterpret_cast<float4*>(x + e) = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const double emax = st->eps_max, den = st->eps_max - st->eps_min;
    const float* h = H + tile * TS;
    for (int e = threadIdx.x; e < B * B; e += 256) {
        const int64_t row = I * B + e / B, col = K * B + e % B;
        double v = 0.0;
        if (row < n && col < n) v = ((row == col ? emax : 0.0) - (double)h[e]) / den;
        x[e] = (float)v;
    }
}

// One wave per tile: squared norm in the fixed order (per column over rows
// with FMA, then the pairwise column tree), tile exponent, diagonal sum.
template <int B>
__global__ void __launch_bounds__(64) k_tile_stats(const float* __restrict__ T, const double* __restrict__ SH,
                                                   int64_t nb, double* __restrict__ S, int8_t* __restrict__ texp,
                                                   double* __restrict__ diag) {
    const int64_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    if (tile / nb != tile % nb && SH[tile] == 0.0) {  // the zeros written by k_sp2_init_x
        if (lane == 0) {
            S[tile] = 0.0;
            texp[tile] = (int8_t)-128;
        }
        return;
    }
    const float* t = T + tile * (int64_t)B * B;
    double s = 0.0, mx = 0.0, dv = 0.0;
    if (B == 128) {
        double s2 = 0.0;
        for (int r = 0; r < B; ++r) {
            const double a0 = t[r * B + lane], a1 = t[r * B + lane + 64];
            s = __fma_rn(a0, a0, s);
            s2 = __fma_rn(a1, a1, s2);
            mx = fmax(mx, fmax(fabs(a0), fabs(a1)));
        }
        s = s + s2;
        dv = (double)t[lane * B + lane] + (double)t[(lane + 64) * B + lane + 64];
    } else if (lane < B) {
        for (int r = 0; r < B; ++r) {
            const double a0 = t[r * B + lane];
            s = __fma_rn(a0, a0, s);
            mx = fmax(mx, fabs(a0));
        }
        dv = t[lane * B + lane];
    }
    constexpr int H0 = (B == 128 ? 64 : B) / 2;
    for (int h = H0; h >= 1; h >>= 1) {
        const double o = __shfl_down(s, h, 64);
        if (lane < h) s = s + o;
    }
    for (int h = 32; h >= 1; h >>= 1) {
        const double o = __shfl_down(dv, h, 64);
        if (lane < h) dv = dv + o;
        mx = fmax(mx, __shfl_xor(mx, h, 64));
    }
    if (lane == 0) {
        S[tile] = s;
        int e = -128;
        if (mx > 0.0) {
            e = ilogb(mx);
            e = e < -127 ? -127 : (e > 127 ? 127 : e);
        }
        if (s != s) e = 127;  // fmax passed over a NaN, the norm did not: not known zero
        texp[tile] = (int8_t)e;
        const int64_t I = tile / nb, K = tile % nb;
        if (I == K) diag[nb * nb + I] = dv;
    }
}

__global__ void __launch_bounds__(1024) k_sp2_start(const double* part, int64_t nb, Sp2State* st) {
    __shared__ double red[1024];
    const double tr = block_sum_fixed(part + nb * nb, nb, red);
    if (threadIdx.x == 0) {
        st->cur_trace = tr;
        st->branch = tr > st->n_occ ? 0 : 1;
        st->active = 1;
        st->iter = 0;
        st->converged = 0;
        st->stagnated = 0;
        st->result_step = 0;
        st->list_count = 0;
        st->fin_ticket = 0;
    }
}

// After step m: e_m from the per-tile partials, tr(X_{m+1}) from the diagonal
// partials, the stop rules, and the branch of step m+1.  kFinBlocks blocks
// each add a fixed contiguous range of the nb^2 partials in a fixed order;
// the last block to finish (device-scope fence, then a ticket it resets)
// adds the block sums in a fixed order, so the sums do not depend on timing.
constexpr int kFinBlocks = 64;
constexpr int kFinThreads = 256;

__device__ double block_tree_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int h = kFinThreads / 2; h >= 1; h >>= 1) {
        if (t < h) red[t] = red[t] + red[t + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kFinThreads) k_sp2_finalize(const double* part, int64_t nb,
                                                              unsigned long long* survivors0, Sp2State* st,
                                                              int m, double* bsum, unsigned* ticket) {
    if (st->active == 0) return;  // read by every block before the last one writes it
    __shared__ double red[kFinThreads];
    __shared__ int s_last;
    const int t = threadIdx.x;
    const int64_t cnt = nb * nb;
    const int64_t per = (cnt + kFinBlocks - 1) / kFinBlocks;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < cnt ? lo + per : cnt;
    double s = 0.0;
    for (int64_t i = lo + t; i < hi; i += kFinThreads) s += part[i];
    s = block_tree_sum(s, red);
    if (t == 0) {
        bsum[blockIdx.x] = s;
        __threadfence();
        s_last = atomicAdd(ticket, 1u) == kFinBlocks - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const double e2 = block_tree_sum(t < kFinBlocks ? bsum[t] : 0.0, red);
    double d = 0.0;
    for (int64_t i = t; i < nb; i += kFinThreads) d += part[cnt + i];
    const double tr_next = block_tree_sum(d, red);
    if (t != 0) return;
    *ticket = 0u;
    const double e = sqrt(e2);
    st->trace[m] = st->cur_trace;
    st->idem[m] = e;
    st->br[m] = st->branch;
    st->tasks[m] = *survivors0;
    *survivors0 = 0;  // the next step's cull counts afresh (it may run without a zeroing launch)
    st->iter = m + 1;
    st->list_count = 0;  // the next step lists its tiles afresh
    if (e <= st->tol) {
        st->converged = 1;
        st->result_step = m + 1;
        st->active = 0;
        st->cur_trace = tr_next;
        return;
    }
    if (m >= 2 && st->idem[m - 2] < kStagBelow && e >= st->idem[m - 2]) {
        st->stagnated = 1;
        st->result_step = m;
        st->active = 0;
        return;
    }
    st->cur_trace = tr_next;
    st->branch = tr_next > st->n_occ ? 0 : 1;
    st->result_step = m + 1;
    if (m + 1 >= st->max_iter) st->active = 0;
}

// E = tr(P H) = sum over tiles (I,K) of <P_IK, (H_KI)^T>, one block per tile.
// A pair with a zero tile (squared norm 0: every element is zero) adds
// exactly 0 and is not read; otherwise H_KI is staged in LDS, so both tiles
// are read along their rows, and the block adds the exact FP64 products.
template <int B>
__global__ void __launch_bounds__(256) k_energy_tiles(const float* __restrict__ P, const float* __restrict__ H,
                                                      const double* __restrict__ SP, const double* __restrict__ SH,
                                                      int64_t nb, double* __restrict__ out) {
    __shared__ float hs[B][B + 1];
    __shared__ double red[4];
    const int64_t tile = blockIdx.x;
    const int64_t I = tile / nb, K = tile % nb;
    const int64_t th = K * nb + I;
    if (SP[tile] == 0.0 || SH[th] == 0.0) {
        if (threadIdx.x == 0) out[tile] = 0.0;
        return;
    }
    const float* p = P + tile * (int64_t)B * B;
    const float* h = H + th * (int64_t)B * B;
    for (int e = threadIdx.x; e < B * B; e += 256) hs[e / B][e % B] = h[e];
    __syncthreads();
    double s = 0.0;
    for (int e = threadIdx.x; e < B * B; e += 256) {
        const int r = e / B, c = e % B;
        s = __fma_rn((double)p[e], (double)hs[c][r], s);
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_down(s, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[tile] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The C tiles step m must write: those with a kept product, those whose X
// tile is non-zero (2X - X^2 needs it), and those whose stored values are
// not already known to be zero (exponent -128).  Every other tile keeps its
// zeros and zero norm, and gets zero SP2 partials here.  The list order
// depends on the atomics; each tile's result does not.
__global__ void __launch_bounds__(256) k_sp2_tiles(const ProdDesc* __restrict__ desc, uint32_t* __restrict__ list,
                                                   Sp2State* st, const int* active) {
    if (active && *active == 0) return;
    const ProdDesc& d = *desc;
    const int64_t nb = d.nb, tiles = nb * nb;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool need = false;
    // symmetric squaring: a tile below the diagonal is written (values,
    // norm, exponent, partial) by its mirror above, so it is never listed
    const int64_t I = t / nb, J = t % nb;
    if (t < tiles && !(d.sym_upper && I > J)) {
        const int64_t mirror = J * nb + I;
        uint64_t any = 0;
        for (int k = 0; k < d.W; ++k) any |= d.mask[t * d.W + k];
        need = any != 0 || d.SA[t] != 0.0 || d.eC[t] != -128 || (d.sym_upper && I < J && d.eC[mirror] != -128);
        if (!need) {
            d.sp2_part[t] = 0.0;
            if (I == J) d.sp2_part[tiles + I] = 0.0;
            if (d.sym_upper && I < J) d.sp2_part[mirror] = 0.0;
        }
    }
    const unsigned long long m = __ballot(need);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(&st->list_count, (unsigned)__popcll(m));
    base = (unsigned)__shfl((int)base, 0, 64);
    if (need) list[base + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)t;
}

// Exact symmetry of H, one block per tile pair (I <= J): element (r, c) of
// tile (I, J) equals element (c, r) of tile (J, I).  Pairs of zero tiles
// (both squared norms 0) are not read.
__global__ void __launch_bounds__(256) k_check_symmetric(const float* __restrict__ T, const double* __restrict__ S,
                                                         int64_t nb, int b, unsigned* flag) {
    const int64_t t = blockIdx.x;
    const int64_t I = t / nb, J = t % nb;
    if (I > J) return;
    if (S[I * nb + J] == 0.0 && S[J * nb + I] == 0.0) return;
    const int64_t ts = (int64_t)b * b;
    const float* a = T + (I * nb + J) * ts;
    const float* m = T + (J * nb + I) * ts;
    bool bad = false;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e / b, c = e % b;
        bad |= !(a[e] == m[c * b + r]) && !(a[e] != a[e] && m[c * b + r] != m[c * b + r]);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ void __launch_bounds__(1024) k_sum_to(const double* x, int64_t count, double* out) {
    __shared__ double red[1024];
    const double s = block_sum_fixed(x, count, red);
    if (threadIdx.x == 0) *out = s;
}

__global__ void k_trace_of(const double* part, int64_t nb, double* out) {
    __shared__ double red[1024];
    const double s = block_sum_fixed(part + nb * nb, nb, red);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

hipError_t launch_sp2_tiles(const ProdDesc* d_desc, int64_t nb, uint32_t* list, Sp2State* st, const int* active,
                            hipStream_t s) {
    const int64_t tiles = nb * nb;
    hipLaunchKernelGGL(k_sp2_tiles, dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, s, d_desc, list, st, active);
    return hipGetLastError();
}

hipError_t launch_check_symmetric(const spamm_matrix* H, unsigned* flag, hipStream_t s) {
    if (H->dt != SPAMM_F32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_check_symmetric, dim3((unsigned)(H->nb * H->nb)), dim3(256), 0, s, (const float*)H->tiles,
                       H->norms, H->nb, H->b, flag);
    return hipGetLastError();
}

hipError_t launch_gershgorin(const spamm_matrix* H, double* lo, double* hi, Sp2State* st, hipStream_t s) {
    hipLaunchKernelGGL(k_gersh_rows, dim3((unsigned)((H->n + 3) / 4)), dim3(256), 0, s, (const float*)H->tiles,
                       H->norms, H->n, H->b, H->nb, lo, hi);
    hipLaunchKernelGGL(k_gersh_reduce, dim3(1), dim3(1024), 0, s, lo, hi, H->n, st);
    return hipGetLastError();
}

hipError_t launch_sp2_init(const spamm_matrix* H, spamm_matrix* X, double* part, Sp2State* st, hipStream_t s) {
    const unsigned tiles = (unsigned)(X->nb * X->nb);
    const float* ht = (const float*)H->tiles;
    float* xt = (float*)X->tiles;
    switch (X->b) {
        case 32:
            hipLaunchKernelGGL(k_sp2_init_x<32>, dim3(tiles), dim3(256), 0, s, ht, H->norms, xt, H->n, H->nb, st);
            hipLaunchKernelGGL(k_tile_stats<32>, dim3(tiles), dim3(64), 0, s, xt, H->norms, X->nb, X->norms, X->texp, part);
            break;
        case 64:
            hipLaunchKernelGGL(k_sp2_init_x<64>, dim3(tiles), dim3(256), 0, s, ht, H->norms, xt, H->n, H->nb, st);
            hipLaunchKernelGGL(k_tile_stats<64>, dim3(tiles), dim3(64), 0, s, xt, H->norms, X->nb, X->norms, X->texp, part);
            break;
        case 128:
            hipLaunchKernelGGL(k_sp2_init_x<128>, dim3(tiles), dim3(256), 0, s, ht, H->norms, xt, H->n, H->nb, st);
            hipLaunchKernelGGL(k_tile_stats<128>, dim3(tiles), dim3(64), 0, s, xt, H->norms, X->nb, X->norms, X->texp, part);
            break;
        default: return hipErrorInvalidValue;
    }
    X->tiers_valid = false;  // X_0's upper tiers are formed if a product reads them
    hipLaunchKernelGGL(k_sp2_start, dim3(1), dim3(1024), 0, s, part, X->nb, st);
    return hipGetLastError();
}

namespace {

#ifndef GLOBAL
#define GLOBAL __attribute__((address_space(1)))
#endif
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Block dropping of the new iterate (section 3, scheme I): one wave per tile.
// A tile whose squared norm (from the epilogue that wrote it) is below tau2
// and that is not already known to be zero is zeroed, with its norm, its
// exponent and, on the diagonal, its trace partial.  Its idempotency partial
// stays: it measures the step's product, not the filtered iterate.
template <int B>
__global__ void __launch_bounds__(256) k_sp2_drop(float* __restrict__ X, double* __restrict__ S,
                                                  int8_t* __restrict__ ex, double* __restrict__ part, int64_t nb,
                                                  double tau2, const int* __restrict__ active) {
    if (active && *active == 0) return;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= nb * nb) return;
    const int lane = threadIdx.x & 63;
    if (!(S[t] < tau2) || ex[t] == -128) return;  // (the same words in every lane of the wave)
    GLOBAL f32x4* x = (GLOBAL f32x4*)(X + t * (int64_t)B * B);
    for (int u = lane; u < B * B / 4; u += 64) x[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (lane == 0) {
        S[t] = 0.0;
        ex[t] = (int8_t)-128;
        if (t / nb == t % nb) part[nb * nb + t / nb] = 0.0;
    }
}

}  // namespace

hipError_t launch_sp2_drop(spamm_matrix* X, double* part, double tau2, const int* active, hipStream_t s) {
    const int64_t tiles = X->nb * X->nb;
    const unsigned blocks = (unsigned)((tiles + 3) / 4);
    switch (X->b) {
        case 32:
            hipLaunchKernelGGL(k_sp2_drop<32>, dim3(blocks), dim3(256), 0, s, (float*)X->tiles, X->norms, X->texp,
                               part, X->nb, tau2, active);
            break;
        case 64:
            hipLaunchKernelGGL(k_sp2_drop<64>, dim3(blocks), dim3(256), 0, s, (float*)X->tiles, X->norms, X->texp,
                               part, X->nb, tau2, active);
            break;
        case 128:
            hipLaunchKernelGGL(k_sp2_drop<128>, dim3(blocks), dim3(256), 0, s, (float*)X->tiles, X->norms, X->texp,
                               part, X->nb, tau2, active);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sp2_finalize(const double* part, int64_t nb, unsigned long long* survivors0, Sp2State* st,
                               int m, hipStream_t s) {
    hipLaunchKernelGGL(k_sp2_finalize, dim3(kFinBlocks), dim3(kFinThreads), 0, s, part, nb, survivors0, st, m,
                       st->fin_bsum, &st->fin_ticket);
    return hipGetLastError();
}

hipError_t launch_energy(const spamm_matrix* P, const spamm_matrix* H, double* tile_part, double* out,
                         hipStream_t s) {
    const int64_t tiles = P->nb * P->nb;
    const float* pt = (const float*)P->tiles;
    const float* ht = (const float*)H->tiles;
    switch (P->b) {
        case 32: hipLaunchKernelGGL(k_energy_tiles<32>, dim3((unsigned)tiles), dim3(256), 0, s, pt, ht, P->norms, H->norms, P->nb, tile_part); break;
        case 64: hipLaunchKernelGGL(k_energy_tiles<64>, dim3((unsigned)tiles), dim3(256), 0, s, pt, ht, P->norms, H->norms, P->nb, tile_part); break;
        case 128: hipLaunchKernelGGL(k_energy_tiles<128>, dim3((unsigned)tiles), dim3(256), 0, s, pt, ht, P->norms, H->norms, P->nb, tile_part); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(1024), 0, s, tile_part, tiles, out);
    return hipGetLastError();
}

}  // namespace spamm
