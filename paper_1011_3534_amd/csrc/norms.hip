// Quadtree construction on gfx950: packing into b x b tiles, the FP64 leaf
// norms in their fixed summation order, and the upper tiers (section 2,
// Eq. 1; Frobenius norm as in section 3).
//
// One wavefront owns a strip of b rows by 64*V columns (V elements of 16
// bytes per lane), so each row of the strip is one 1 KiB coalesced load and
// each lane streams its V columns down all b rows, accumulating x*x with a
// fused multiply-add in FP64 (exact for FP32 inputs).  The column sums of a
// tile are then combined by the pairwise tree s_c += s_{c+h}, h = b/2 .. 1,
// across lanes (shuffles) and finally inside a lane.
#include <algorithm>
#include <cstring>

#include "spamm_internal.hpp"

namespace spamm {
namespace {

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int V = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int V = 2;
};

__device__ inline double shfl_down_d(double v, int d) { return __shfl_down(v, d, kWave); }
__device__ inline float shfl_xor_f(float v, int d) { return __shfl_xor(v, d, kWave); }

// Exponent e with max|x| in [2^e, 2^(e+1)); -128 for an all-zero tile.  The
// maximum (fmax) passes over NaN, but the tile's squared norm S does not: a
// NaN anywhere makes S NaN, and the tile then gets 127 ("not known zero",
// as for inf), never the all-zero mark.
__device__ inline int8_t tile_exponent(double mx, double S) {
    if (S != S) return (int8_t)127;
    if (!(mx > 0.0)) return (int8_t)-128;
    int e = ilogb(mx);
    e = e < -127 ? -127 : (e > 127 ? 127 : e);
    return (int8_t)e;
}

// Wave gw of one matrix: tile row I = gw / nstrips, column strip gw % nstrips.
template <typename T, int B>
__device__ __forceinline__ void pack_wave(const T* __restrict__ a, int64_t n, int64_t lda, int64_t nb,
                                          int64_t nstrips, T* __restrict__ tiles, double* __restrict__ S0,
                                          int8_t* __restrict__ texp, int vec, int64_t gw) {
    constexpr int V = Vec16<T>::V;
    constexpr int LPT = B / V;  // lanes per tile
    using VT = typename Vec16<T>::type;
    const int lane = threadIdx.x & (kWave - 1);
    if (gw >= nb * nstrips) return;
    const int64_t I = gw / nstrips;
    const int64_t s = gw % nstrips;
    const int64_t col = s * (int64_t)(kWave * V) + (int64_t)lane * V;
    const int64_t K = col / B;
    const int cin = (int)(col % B);
    const bool live = K < nb;

    double acc[V];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < V; ++j) acc[j] = 0.0;

    // (a view keeps the caller's array as its tiles: tiles == NULL, norms only)
    T* tdst = tiles ? tiles + ((I * nb + (live ? K : 0)) * B) * (int64_t)B + cin : nullptr;
    // 16 rows of loads in flight per wave (a norms-only pass reads at 6.3
    // TB/s with 16, 5.9 with 8; deeper unrolling slows the packing pass)
#pragma unroll 16
    for (int r = 0; r < B; ++r) {
        const int64_t row = I * B + r;
        T x[V];
        if (vec) {
            if (row < n && col < n) {
                VT v = *reinterpret_cast<const VT*>(a + row * lda + col);
                const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
                for (int j = 0; j < V; ++j) x[j] = pv[j];
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) x[j] = (T)0;
            }
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) x[j] = (row < n && col + j < n) ? a[row * lda + col + j] : (T)0;
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            double xd = (double)x[j];
            acc[j] = __fma_rn(xd, xd, acc[j]);
            mx = fmax(mx, fabs(xd));
        }
        if (live && tiles) {
            VT v;
            T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
            for (int j = 0; j < V; ++j) pv[j] = x[j];
            *reinterpret_cast<VT*>(tdst + (int64_t)r * B) = v;
        }
    }
    // pairwise tree over the b columns of the tile: first across lanes ...
    const int tl = lane % LPT;
#pragma unroll
    for (int h = B / 2; h >= V; h /= 2) {
        const int d = h / V;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            double o = shfl_down_d(acc[j], d);
            if (tl < d) acc[j] = acc[j] + o;
        }
    }
    // ... then inside the lane
#pragma unroll
    for (int h = V / 2; h >= 1; h /= 2)
#pragma unroll
        for (int c = 0; c < h; ++c) acc[c] = acc[c] + acc[c + h];
    // tile max |x| for the power-of-two scaling of 16-bit leaves
#pragma unroll
    for (int d = 1; d < LPT; d *= 2) mx = fmax(mx, (double)__shfl_xor(mx, d, kWave));
    if (live && tl == 0) {
        S0[I * nb + K] = acc[0];
        texp[I * nb + K] = tile_exponent(mx, acc[0]);
    }
}

template <typename T, int B>
__global__ void __launch_bounds__(256) k_pack_norm(const T* __restrict__ a, int64_t n, int64_t lda,
                                                   int64_t nb, int64_t nstrips, T* __restrict__ tiles,
                                                   double* __restrict__ S0, int8_t* __restrict__ texp,
                                                   int vec) {
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    pack_wave<T, B>(a, n, lda, nb, nstrips, tiles, S0, texp, vec, gw);
}

// Batch: the waves of all matrices in one launch; wave_base is the first
// global wave of each matrix (ascending), so a binary search finds the matrix.
template <typename T, int B>
__global__ void __launch_bounds__(256) k_pack_norm_batched(const PackDesc* __restrict__ pd, int count) {
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pd[mid].wave_base <= gw) lo = mid; else hi = mid - 1;
    }
    const PackDesc& d = pd[lo];
    pack_wave<T, B>((const T*)d.a, d.n, d.lda, d.nb, d.nstrips, (T*)d.tiles, d.S0, d.texp, d.vec,
                    gw - d.wave_base);
}

// One tier up: P[I,K] = (S[2I,2K] + S[2I,2K+1]) + (S[2I+1,2K] + S[2I+1,2K+1]).
__global__ void k_norm_parent(const double* __restrict__ S, int m, double* __restrict__ P, int mp,
                              const int* active) {
    if (active && *active == 0) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)mp * mp) return;
    const int I = (int)(t / mp), K = (int)(t % mp);
    double c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 2 * I + (q >> 1), k = 2 * K + (q & 1);
        c[q] = (i < m && k < m) ? S[(int64_t)i * m + k] : 0.0;
    }
    P[t] = (c[0] + c[1]) + (c[2] + c[3]);
}

constexpr int kSmallTier = 64;  // tiers with m_l <= kSmallTier go to the single-block kernels

// Batch, one large tier l for every matrix (blockIdx.y) that has it.
__global__ void k_norm_parent_batched(const NormTable* __restrict__ tab, int l) {
    const NormTable& t = tab[blockIdx.y];
    if (l > t.L) return;
    const int m = t.m[l - 1], mp = t.m[l];
    if (mp <= kSmallTier) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)mp * mp) return;
    const double* S = t.norms + t.off[l - 1];
    const int I = (int)(i / mp), K = (int)(i % mp);
    double c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 2 * I + (q >> 1), k = 2 * K + (q & 1);
        c[q] = (r < m && k < m) ? S[(int64_t)r * m + k] : 0.0;
    }
    t.norms[t.off[l] + i] = (c[0] + c[1]) + (c[2] + c[3]);
}

// The small tiers l0 .. L of one pyramid in one block, tier by tier.  Only
// the first tier reads its children from global memory; every tier is kept
// in LDS (two buffers in turn: tier l0 has at most kSmallTier^2 nodes, the
// next a quarter of that) for the next one, and written to global memory
// once, so the chain of tiers waits on LDS rather than on global round trips.
// The sum of each node is the same 2 x 2 pairwise sum as everywhere else.
constexpr int kSmallThreads = 1024;

template <typename OFF, typename MM>
__device__ void small_tiers(double* __restrict__ norms, const OFF& off, const MM& mm, int l0, int L, double* buf0,
                            double* buf1) {
    // tier l0 from global memory: every load of a thread is issued before
    // its first store (the loads and stores share the pyramid, so the
    // compiler would otherwise wait for each node's children in turn)
    {
        constexpr int U = kSmallTier * kSmallTier / kSmallThreads;
        const double* S = norms + off[l0 - 1];
        double* P = norms + off[l0];
        const int m = mm[l0 - 1], mp = mm[l0];
        double c[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = threadIdx.x + u * kSmallThreads;
            const int I = t / mp, K = t % mp;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 2 * I + (q >> 1), k = 2 * K + (q & 1);
                c[u][q] = (t < mp * mp && i < m && k < m) ? S[(int64_t)i * m + k] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = threadIdx.x + u * kSmallThreads;
            if (t < mp * mp) {
                const double v = (c[u][0] + c[u][1]) + (c[u][2] + c[u][3]);
                buf0[t] = v;
                P[t] = v;
            }
        }
        __syncthreads();
    }
    const double* src = buf0;
    for (int l = l0 + 1; l <= L; ++l) {
        double* dst = ((l - l0) & 1) ? buf1 : buf0;
        double* P = norms + off[l];
        const int m = mm[l - 1], mp = mm[l];
        for (int t = threadIdx.x; t < mp * mp; t += blockDim.x) {
            const int I = t / mp, K = t % mp;
            double c[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 2 * I + (q >> 1), k = 2 * K + (q & 1);
                c[q] = (i < m && k < m) ? src[(int64_t)i * m + k] : 0.0;
            }
            const double v = (c[0] + c[1]) + (c[2] + c[3]);
            dst[t] = v;
            P[t] = v;
        }
        __syncthreads();
        src = dst;
    }
}

// Batch, the small tiers of matrix blockIdx.x in one block.
__global__ void __launch_bounds__(kSmallThreads) k_norm_small_tiers_batched(const NormTable* __restrict__ tab) {
    __shared__ double buf0[kSmallTier * kSmallTier], buf1[kSmallTier * kSmallTier / 4];
    const NormTable& t = tab[blockIdx.x];
    int l0 = 1;
    while (l0 <= t.L && t.m[l0] > kSmallTier) ++l0;
    if (l0 <= t.L) small_tiers(t.norms, t.off, t.m, l0, t.L, buf0, buf1);
}

// The small upper tiers of one pyramid in one block.
__global__ void __launch_bounds__(kSmallThreads) k_norm_small_tiers(double* __restrict__ norms, const int64_t* off,
                                                           const int* mm, int l0, int L, const int* active) {
    if (active && *active == 0) return;
    __shared__ double buf0[kSmallTier * kSmallTier], buf1[kSmallTier * kSmallTier / 4];
    small_tiers(norms, off, mm, l0, L, buf0, buf1);
}

template <typename T>
__global__ void k_to_dense(const T* __restrict__ tiles, TileGeo g, int64_t n, T* __restrict__ out, int64_t ldo) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = t / n, col = t % n;
    if (row >= n) return;
    out[row * ldo + col] = tiles[g.at(row, col)];
}

template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_diff_norms(const TX* __restrict__ x, const TY* __restrict__ y,
                                                    int64_t count, double* __restrict__ out) {
    double d2 = 0.0, r2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double yv = (double)y[i];
        const double dv = (double)x[i] - yv;
        d2 = __fma_rn(dv, dv, d2);
        r2 = __fma_rn(yv, yv, r2);
    }
    for (int d = kWave / 2; d >= 1; d /= 2) {
        d2 += __shfl_down(d2, d, kWave);
        r2 += __shfl_down(r2, d, kWave);
    }
    __shared__ double sd[4], sr[4];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sd[w] = d2;
        sr[w] = r2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b2 = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
            a += sd[i];
            b2 += sr[i];
        }
        out[2 * blockIdx.x] = a;
        out[2 * blockIdx.x + 1] = b2;
    }
}

// ||X - Y||^2 and ||Y||^2 for handles of equal n but different layouts
// (leaf sizes, views): element (row, col) is looked up in each handle's own.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_diff_norms_any(const TX* __restrict__ x, TileGeo gx,
                                                        const TY* __restrict__ y, TileGeo gy, int64_t n,
                                                        double* __restrict__ out) {
    double d2 = 0.0, r2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / n, col = i % n;
        const double xv = (double)x[gx.at(row, col)];
        const double yv = (double)y[gy.at(row, col)];
        const double dv = xv - yv;
        d2 = __fma_rn(dv, dv, d2);
        r2 = __fma_rn(yv, yv, r2);
    }
    for (int d = kWave / 2; d >= 1; d /= 2) {
        d2 += __shfl_down(d2, d, kWave);
        r2 += __shfl_down(r2, d, kWave);
    }
    __shared__ double sd[4], sr[4];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sd[w] = d2;
        sr[w] = r2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = (sd[0] + sd[1]) + (sd[2] + sd[3]);
        out[2 * blockIdx.x + 1] = (sr[0] + sr[1]) + (sr[2] + sr[3]);
    }
}

__global__ void k_fill_u64(uint64_t* p, int64_t count, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T, int B>
hipError_t pack_t(const void* a, int64_t n, int64_t lda, spamm_matrix* M, hipStream_t s) {
    constexpr int V = Vec16<T>::V;
    const int64_t nb = M->nb;
    const int64_t nstrips = (nb * B + kWave * V - 1) / (kWave * V);
    const int64_t waves = nb * nstrips;
    const int64_t blocks = (waves + 3) / 4;
    const int vec = ((uintptr_t)a % 16 == 0) && (lda % V == 0) && (n % V == 0);
    hipLaunchKernelGGL((k_pack_norm<T, B>), dim3((unsigned)blocks), dim3(256), 0, s, (const T*)a, n, lda, nb,
                       nstrips, M->view ? nullptr : (T*)M->tiles, M->norms, M->texp, vec);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_norm(const void* a, int64_t n, int64_t lda, spamm_dtype dt, spamm_matrix* M,
                            int split_kind, hipStream_t s) {
    if (split_kind >= 0) {
        // pack, then split the tiles just written (measured faster than one
        // fused pass that keeps each column's values in registers)
        if (dt != SPAMM_F32 || !M->split) return hipErrorInvalidValue;
        hipError_t e = hipErrorInvalidValue;
        switch (M->b) {
            case 32: e = pack_t<float, 32>(a, n, lda, M, s); break;
            case 64: e = pack_t<float, 64>(a, n, lda, M, s); break;
            case 128: e = pack_t<float, 128>(a, n, lda, M, s); break;
        }
        return e == hipSuccess ? launch_split(M, split_kind, nullptr, s) : e;
    }
    if (dt == SPAMM_F32) {
        switch (M->b) {
            case 32: return pack_t<float, 32>(a, n, lda, M, s);
            case 64: return pack_t<float, 64>(a, n, lda, M, s);
            case 128: return pack_t<float, 128>(a, n, lda, M, s);
        }
    } else {
        switch (M->b) {
            case 32: return pack_t<double, 32>(a, n, lda, M, s);
            case 64: return pack_t<double, 64>(a, n, lda, M, s);
            case 128: return pack_t<double, 128>(a, n, lda, M, s);
        }
    }
    return hipErrorInvalidValue;
}

// Upper tiers: one launch per large tier, then the small ones in one block.
hipError_t launch_upper_norms(spamm_matrix* M, hipStream_t s, const int* active) {
    constexpr int kSmall = kSmallTier;
    int l = 1;
    for (; l <= M->L && M->lvl_m[l] > kSmall; ++l) {
        const int m = M->lvl_m[l - 1], mp = M->lvl_m[l];
        const int64_t cnt = (int64_t)mp * mp;
        hipLaunchKernelGGL(k_norm_parent, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           M->norms + M->lvl_off[l - 1], m, M->norms + M->lvl_off[l], mp, active);
    }
    if (l <= M->L) {
        // tier offsets/sizes travel as kernel arguments through a small device table
        // kept at the end of the pyramid allocation
        int64_t* off = reinterpret_cast<int64_t*>(M->norms + M->norms_total);
        int* mm = reinterpret_cast<int*>(off + kMaxLevels);
        hipLaunchKernelGGL(k_norm_small_tiers, dim3(1), dim3(kSmallThreads), 0, s, M->norms, off, mm, l, M->L, active);
    }
    return hipGetLastError();
}

NormTable norm_table(const spamm_matrix* M) {
    NormTable t;
    std::memset(&t, 0, sizeof t);
    t.norms = M->norms;
    for (int l = 0; l < kMaxLevels; ++l) {
        t.off[l] = M->lvl_off[l];
        t.m[l] = M->lvl_m[l];
    }
    t.L = M->L;
    return t;
}

// Upper tiers of count handles: one launch per large tier for all of them,
// then one block per handle for its small tiers.  d_tab: count device tables
// (filled by the caller from norm_table).
hipError_t launch_upper_norms_batched(spamm_matrix* const* M, int count, const NormTable* d_tab, hipStream_t s) {
    int Lmax = 0;
    for (int m = 0; m < count; ++m) Lmax = std::max(Lmax, M[m]->L);
    for (int l = 1; l <= Lmax; ++l) {
        int64_t cells = 0;
        for (int m = 0; m < count; ++m)
            if (l <= M[m]->L && M[m]->lvl_m[l] > kSmallTier)
                cells = std::max<int64_t>(cells, (int64_t)M[m]->lvl_m[l] * M[m]->lvl_m[l]);
        if (cells == 0) break;
        hipLaunchKernelGGL(k_norm_parent_batched, dim3((unsigned)((cells + 255) / 256), (unsigned)count), dim3(256), 0,
                           s, d_tab, l);
    }
    hipLaunchKernelGGL(k_norm_small_tiers_batched, dim3((unsigned)count), dim3(kSmallThreads), 0, s, d_tab);
    return hipGetLastError();
}

// One pack launch for count matrices of one element type and leaf size;
// d_pd: count device descriptors (filled by the caller from pack_desc, in
// order, so wave_base ascends).
hipError_t launch_pack_norm_batched(const PackDesc* d_pd, int count, int64_t waves, spamm_dtype dt, int b,
                                    hipStream_t s) {
    const unsigned blocks = (unsigned)((waves + 3) / 4);
#define SPAMM_PACK_B(T, BB) \
    hipLaunchKernelGGL((k_pack_norm_batched<T, BB>), dim3(blocks), dim3(256), 0, s, d_pd, count)
    if (dt == SPAMM_F32) {
        switch (b) {
            case 32: SPAMM_PACK_B(float, 32); break;
            case 64: SPAMM_PACK_B(float, 64); break;
            case 128: SPAMM_PACK_B(float, 128); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (b) {
            case 32: SPAMM_PACK_B(double, 32); break;
            case 64: SPAMM_PACK_B(double, 64); break;
            case 128: SPAMM_PACK_B(double, 128); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef SPAMM_PACK_B
    return hipGetLastError();
}

// Descriptor of one matrix of a batched pack; wave_base as laid out by the caller.
PackDesc pack_desc(const void* a, int64_t n, int64_t lda, spamm_matrix* M, int64_t wave_base) {
    PackDesc d;
    std::memset(&d, 0, sizeof d);
    const int V = M->dt == SPAMM_F32 ? 4 : 2;
    d.a = a;
    d.n = n;
    d.lda = lda;
    d.nb = M->nb;
    d.nstrips = (M->nb * M->b + kWave * V - 1) / (kWave * V);
    d.wave_base = wave_base;
    d.tiles = M->view ? nullptr : M->tiles;
    d.S0 = M->norms;
    d.texp = M->texp;
    d.vec = ((uintptr_t)a % 16 == 0) && (lda % V == 0) && (n % V == 0);
    return d;
}

hipError_t launch_to_dense(const spamm_matrix* M, void* out, int64_t ldo, hipStream_t s) {
    const int64_t cnt = M->n * M->n;
    const unsigned blocks = (unsigned)((cnt + 255) / 256);
    if (M->dt == SPAMM_F32)
        hipLaunchKernelGGL(k_to_dense<float>, dim3(blocks), dim3(256), 0, s, (const float*)M->tiles, tile_geo(M),
                           M->n, (float*)out, ldo);
    else
        hipLaunchKernelGGL(k_to_dense<double>, dim3(blocks), dim3(256), 0, s, (const double*)M->tiles,
                           tile_geo(M), M->n, (double*)out, ldo);
    return hipGetLastError();
}

// Padding is zero in both packed handles, so their padded tile storage can
// be compared element by element.
hipError_t launch_diff_norms(const spamm_matrix* X, const spamm_matrix* Y, double* d_out, hipStream_t s) {
    const int64_t count = X->nb * X->nb * (int64_t)X->b * X->b;
    const unsigned blocks = 1024;
    const bool xf = X->dt == SPAMM_F32, yf = Y->dt == SPAMM_F32;
    if (X->b != Y->b || X->view || Y->view) {
#define SPAMM_DIFF_ANY(TX, TY)                                                                                   \
    hipLaunchKernelGGL((k_diff_norms_any<TX, TY>), dim3(blocks), dim3(256), 0, s, (const TX*)X->tiles, tile_geo(X), \
                       (const TY*)Y->tiles, tile_geo(Y), X->n, d_out)
        if (xf && yf) SPAMM_DIFF_ANY(float, float);
        else if (xf) SPAMM_DIFF_ANY(float, double);
        else if (yf) SPAMM_DIFF_ANY(double, float);
        else SPAMM_DIFF_ANY(double, double);
#undef SPAMM_DIFF_ANY
        return hipGetLastError();
    }
    if (xf && yf)
        hipLaunchKernelGGL((k_diff_norms<float, float>), dim3(blocks), dim3(256), 0, s, (const float*)X->tiles,
                           (const float*)Y->tiles, count, d_out);
    else if (xf)
        hipLaunchKernelGGL((k_diff_norms<float, double>), dim3(blocks), dim3(256), 0, s, (const float*)X->tiles,
                           (const double*)Y->tiles, count, d_out);
    else if (yf)
        hipLaunchKernelGGL((k_diff_norms<double, float>), dim3(blocks), dim3(256), 0, s, (const double*)X->tiles,
                           (const float*)Y->tiles, count, d_out);
    else
        hipLaunchKernelGGL((k_diff_norms<double, double>), dim3(blocks), dim3(256), 0, s,
                           (const double*)X->tiles, (const double*)Y->tiles, count, d_out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, int64_t count, uint64_t v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

}  // namespace spamm
