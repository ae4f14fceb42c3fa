// Seeded synthetic decay matrices on the device.
//
// The same published counter-based generator as the host-side input module
// (SplitMix64, Steele, Lea and Flood, OOPSLA 2014): h = sm64(sm64(seed) ^
// (i << 32 | j)), u = (h >> 11) 2^-53, and a_ij = round(f(|i-j|) * (lo +
// (hi - lo) u)) with the FP64 decay table f supplied by the caller, so host
// and device draw identical matrices.  No part of the multiply uses this.
#include <vector>

#include "spamm_internal.hpp"

namespace spamm {
namespace {

__device__ inline uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void k_gen_decay(T* __restrict__ out, int64_t n, int64_t ld, const double* __restrict__ table,
                            uint64_t seedkey, double lo, double span, int symmetric, const double* __restrict__ diag) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        uint64_t ci = (uint64_t)i, cj = (uint64_t)j;
        if (symmetric && ci > cj) {
            const uint64_t t = ci;
            ci = cj;
            cj = t;
        }
        const uint64_t h = sm64(seedkey ^ ((ci << 32) | cj));
        const double u = (double)(h >> 11) * 0x1.0p-53;
        const double uu = lo + span * u;
        double v = table[i > j ? i - j : j - i] * uu;
        if (diag && i == j) v = diag[i];
        out[i * ld + j] = (T)v;
    }
}

uint64_t host_sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace
}  // namespace spamm

extern "C" spamm_status spamm_generate_decay(int64_t n, int64_t ld, spamm_dtype dt, const double* host_table,
                                             uint64_t seed, double lo, double hi, int32_t symmetric,
                                             const double* host_diag, void* dev_out, void* stream) {
    using namespace spamm;
    if (n < 1 || ld < n) return set_error(SPAMM_EINVAL, "need n >= 1 and ld >= n");
    if (!host_table || !dev_out) return set_error(SPAMM_EINVAL, "null argument");
    if (dt != SPAMM_F32 && dt != SPAMM_F64) return set_error(SPAMM_EINVAL, "unknown dtype");
    hipStream_t s = (hipStream_t)stream;
    const size_t nt = (size_t)n * (host_diag ? 2 : 1);
    const Allocator al = current_allocator();
    double* d = (double*)raw_alloc(al, nt * sizeof(double), s);
    if (!d) return set_error(SPAMM_ENOMEM, "spamm_generate_decay table allocation failed");
    hipError_t e = hipMemcpyAsync(d, host_table, (size_t)n * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && host_diag) e = hipMemcpyAsync(d + n, host_diag, (size_t)n * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const uint64_t key = host_sm64(seed);
        int64_t blocks = (n * n + 255) / 256;
        blocks = blocks > 65536 ? 65536 : blocks;
        const double* dg = host_diag ? d + n : nullptr;
        if (dt == SPAMM_F32)
            hipLaunchKernelGGL(k_gen_decay<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)dev_out, n, ld, d,
                               key, lo, hi - lo, symmetric, dg);
        else
            hipLaunchKernelGGL(k_gen_decay<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)dev_out, n, ld,
                               d, key, lo, hi - lo, symmetric, dg);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    raw_free(al, d, s);
    if (e != hipSuccess) return hip_error(e, "spamm_generate_decay");
    return SPAMM_OK;
}
