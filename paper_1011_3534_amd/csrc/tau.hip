// Learned threshold selector on gfx950: histogram features of the norm
// pyramids, a 515 -> 128 -> 128 -> 128 -> 1 ReLU network trained with Adam,
// and tau selection with an exact-product check and bisection fallback.
//
// Features: for each operand and tier l = 0..7 from the leaves, the fraction
// of tier-l nodes in bin k = #{j in 1..31 : S < S_root * 1e-j}; then
// log10(target), log2(nb)/10, log2(b)/7.  The network predicts
// y = log10(tau / (||A||_F ||B||_F)).  All network arithmetic is FP32 with
// fixed summation orders (deterministic); features are integer counts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "spamm_internal.hpp"

struct spamm_tau_model {
    float* params = nullptr;  // NPARAM
    float* m = nullptr;       // Adam moments
    float* v = nullptr;
    int64_t t = 0;            // Adam step count
    spamm::Allocator al;      // the allocator pair the weights came from
    hipStream_t last_stream = nullptr;  // stream of the last call that used the weights
};

namespace spamm {
namespace {

constexpr int kBins = 32, kTiers = 8, kHid = SPAMM_TAU_HIDDEN, kIn = SPAMM_TAU_NFEAT;
constexpr int64_t kNParam = SPAMM_TAU_NPARAM;
// correctly rounded decimal thresholds 1e-1 .. 1e-31
__constant__ double kThr[kBins - 1] = {1e-1,  1e-2,  1e-3,  1e-4,  1e-5,  1e-6,  1e-7,  1e-8,  1e-9,  1e-10, 1e-11,
                                       1e-12, 1e-13, 1e-14, 1e-15, 1e-16, 1e-17, 1e-18, 1e-19, 1e-20, 1e-21, 1e-22,
                                       1e-23, 1e-24, 1e-25, 1e-26, 1e-27, 1e-28, 1e-29, 1e-30, 1e-31};

// Layer geometry: offsets of W_k and b_k in the flat parameter vector.
struct Layout {
    int64_t w[4], b[4];
    int in[4], out[4];
};
Layout layout() {
    Layout L;
    const int dims[5] = {kIn, kHid, kHid, kHid, 1};
    int64_t k = 0;
    for (int i = 0; i < 4; ++i) {
        L.in[i] = dims[i];
        L.out[i] = dims[i + 1];
        L.w[i] = k;
        k += (int64_t)dims[i] * dims[i + 1];
        L.b[i] = k;
        k += dims[i + 1];
    }
    return L;
}

// block (op, tier): histogram of the tier's squared norms relative to the root
__global__ void __launch_bounds__(256) k_tau_hist(const double* __restrict__ SA, const double* __restrict__ SB,
                                                  const int64_t* __restrict__ off, const int* __restrict__ mm, int L,
                                                  float* __restrict__ feat) {
    __shared__ unsigned cnt[kBins];
    const int op = blockIdx.x / kTiers, l = blockIdx.x % kTiers;
    const double* S = op == 0 ? SA : SB;
    if (threadIdx.x < kBins) cnt[threadIdx.x] = 0;
    __syncthreads();
    if (l <= L) {
        const double root = S[off[L]];
        const int64_t m = mm[l], cntn = m * m;
        for (int64_t i = threadIdx.x; i < cntn; i += blockDim.x) {
            const double s = S[off[l] + i];
            int k = 0;
            for (int j = 0; j < kBins - 1; ++j) k += (s < root * kThr[j]) ? 1 : 0;
            atomicAdd(&cnt[k], 1u);
        }
        __syncthreads();
        if (threadIdx.x < kBins) feat[op * kTiers * kBins + l * kBins + threadIdx.x] = (float)((double)cnt[threadIdx.x] / (double)cntn);
    } else if (threadIdx.x < kBins) {
        feat[op * kTiers * kBins + l * kBins + threadIdx.x] = 0.0f;
    }
}

__global__ void k_tau_scalars(float* feat, float s0, float s1, float s2) {
    feat[2 * kTiers * kBins + 0] = s0;
    feat[2 * kTiers * kBins + 1] = s1;
    feat[2 * kTiers * kBins + 2] = s2;
}

// Y[r, o] = act(b[o] + sum_i X[r, i] W[i, o]), i ascending
template <bool RELU>
__global__ void k_dense_fwd(const float* __restrict__ X, int64_t N, int nin, const float* __restrict__ W,
                            const float* __restrict__ b, float* __restrict__ Y, int nout) {
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N * nout;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / nout;
        const int o = (int)(idx % nout);
        float s = b[o];
        const float* x = X + r * nin;
        for (int i = 0; i < nin; ++i) s = fmaf(x[i], W[(int64_t)i * nout + o], s);
        Y[idx] = RELU ? fmaxf(s, 0.0f) : s;
    }
}

// dY = 2 (yhat - y) / N; per-block partial sums of the squared residual
__global__ void __launch_bounds__(256) k_mse_grad(const float* __restrict__ yhat, const float* __restrict__ y, int64_t N,
                                                  float* __restrict__ dY, float* __restrict__ part) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        const float d = yhat[r] - y[r];
        dY[r] = 2.0f * d / (float)N;
        s = fmaf(d, d, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dW[i, o] = sum_r X[r, i] dY[r, o]; db[o] = sum_r dY[r, o] (r ascending)
__global__ void k_dense_bwd_w(const float* __restrict__ X, int64_t N, int nin, const float* __restrict__ dY, int nout,
                              float* __restrict__ dW, float* __restrict__ db) {
    const int64_t total = (int64_t)nin * nout + nout;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        if (idx < (int64_t)nin * nout) {
            const int i = (int)(idx / nout), o = (int)(idx % nout);
            for (int64_t r = 0; r < N; ++r) s = fmaf(X[r * nin + i], dY[r * nout + o], s);
            dW[idx] = s;
        } else {
            const int o = (int)(idx - (int64_t)nin * nout);
            for (int64_t r = 0; r < N; ++r) s += dY[r * nout + o];
            db[o] = s;
        }
    }
}

// dX[r, i] = (sum_o dY[r, o] W[i, o]) * [Xact[r, i] > 0]
__global__ void k_dense_bwd_x(const float* __restrict__ dY, int64_t N, int nout, const float* __restrict__ W, int nin,
                              const float* __restrict__ Xact, float* __restrict__ dX) {
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N * nin;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / nin;
        const int i = (int)(idx % nin);
        float s = 0.0f;
        for (int o = 0; o < nout; ++o) s = fmaf(dY[r * nout + o], W[(int64_t)i * nout + o], s);
        dX[idx] = Xact[idx] > 0.0f ? s : 0.0f;
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t count, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

unsigned grid_for(int64_t work) {
    int64_t b = (work + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Activations of one batch: h1, h2, h3 (N x 128), yhat (N); gradients dh (2 x N x 128).
struct Work {
    float* h[3];
    float* yhat;
    float* dy;
    float* dh[2];
    float* part;
    float* grad;
};

size_t work_bytes(int64_t N) { return (size_t)(N * kHid * 5 + 2 * N + 8192 + kNParam) * sizeof(float) + 1024; }

Work carve(void* base, int64_t N) {
    Work w;
    float* p = (float*)base;
    for (int i = 0; i < 3; ++i) {
        w.h[i] = p;
        p += N * kHid;
    }
    w.yhat = p;
    p += N;
    w.dy = p;
    p += N;
    w.dh[0] = p;
    p += N * kHid;
    w.dh[1] = p;
    p += N * kHid;
    w.part = p;
    p += 8192;
    w.grad = p;
    return w;
}

hipError_t forward(const float* P, const float* X, int64_t N, Work& w, hipStream_t s) {
    const Layout L = layout();
    const float* in = X;
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(k_dense_fwd<true>, dim3(grid_for(N * kHid)), dim3(256), 0, s, in, N, L.in[k], P + L.w[k],
                           P + L.b[k], w.h[k], kHid);
        in = w.h[k];
    }
    hipLaunchKernelGGL(k_dense_fwd<false>, dim3(grid_for(N)), dim3(256), 0, s, in, N, kHid, P + L.w[3], P + L.b[3],
                       w.yhat, 1);
    return hipGetLastError();
}

// gradient of the MSE over the batch into w.grad; per-block loss partials in w.part
hipError_t backward(const float* P, const float* X, const float* y, int64_t N, Work& w, unsigned& loss_blocks,
                    hipStream_t s) {
    const Layout L = layout();
    loss_blocks = grid_for(N);
    if (loss_blocks > 8192) loss_blocks = 8192;
    hipLaunchKernelGGL(k_mse_grad, dim3(loss_blocks), dim3(256), 0, s, w.yhat, y, N, w.dy, w.part);
    // output layer
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(grid_for(kHid + 1)), dim3(256), 0, s, w.h[2], N, kHid, w.dy, 1,
                       w.grad + L.w[3], w.grad + L.b[3]);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(grid_for(N * kHid)), dim3(256), 0, s, w.dy, N, 1, P + L.w[3], kHid, w.h[2],
                       w.dh[0]);
    int cur = 0;
    for (int k = 2; k >= 0; --k) {
        const float* xin = k == 0 ? X : w.h[k - 1];
        hipLaunchKernelGGL(k_dense_bwd_w, dim3(grid_for((int64_t)L.in[k] * kHid + kHid)), dim3(256), 0, s, xin, N,
                           L.in[k], w.dh[cur], kHid, w.grad + L.w[k], w.grad + L.b[k]);
        if (k > 0) {
            hipLaunchKernelGGL(k_dense_bwd_x, dim3(grid_for(N * kHid)), dim3(256), 0, s, w.dh[cur], N, kHid, P + L.w[k],
                               kHid, w.h[k - 1], w.dh[cur ^ 1]);
            cur ^= 1;
        }
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace spamm

using namespace spamm;

extern "C" {

spamm_status spamm_tau_model_create(const float* host_params, spamm_tau_model** out) {
    if (!host_params || !out) return set_error(SPAMM_EINVAL, "null argument");
    auto* m = new spamm_tau_model();
    m->al = current_allocator();
    const size_t bytes = (size_t)kNParam * sizeof(float);
    m->params = (float*)raw_alloc(m->al, bytes, nullptr);
    m->m = (float*)raw_alloc(m->al, bytes, nullptr);
    m->v = (float*)raw_alloc(m->al, bytes, nullptr);
    if (!m->params || !m->m || !m->v) {
        spamm_tau_model_free(m);
        return set_error(SPAMM_ENOMEM, "tau model allocation failed");
    }
    // set up on the null stream, where the weights were allocated
    hipError_t e = hipMemcpyAsync(m->params, host_params, bytes, hipMemcpyHostToDevice, nullptr);
    if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, bytes, nullptr);
    if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, bytes, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        spamm_tau_model_free(m);
        return hip_error(e, "spamm_tau_model_create");
    }
    *out = m;
    return SPAMM_OK;
}

spamm_status spamm_tau_model_params(const spamm_tau_model* m, float* host_params) {
    if (!m || !host_params) return set_error(SPAMM_EINVAL, "null argument");
    // the weights were last written on last_stream: copy in that stream's order
    SPAMM_HIP(hipMemcpyAsync(host_params, m->params, (size_t)kNParam * sizeof(float), hipMemcpyDeviceToHost,
                             m->last_stream));
    SPAMM_HIP(hipStreamSynchronize(m->last_stream));
    return SPAMM_OK;
}

void spamm_tau_model_free(spamm_tau_model* m) {
    if (!m) return;
    if (m->last_stream) (void)hipStreamSynchronize(m->last_stream);
    raw_free(m->al, m->params, m->last_stream);
    raw_free(m->al, m->m, m->last_stream);
    raw_free(m->al, m->v, m->last_stream);
    delete m;
}

spamm_status spamm_tau_features(const spamm_matrix* A, const spamm_matrix* B, double target, float* dev_out,
                                void* stream) {
    if (!A || !B || !dev_out) return set_error(SPAMM_EINVAL, "null argument");
    if (A->n != B->n || A->b != B->b) return set_error(SPAMM_EINVAL, "operands differ in n or leaf size");
    if (!(target > 0.0) || !std::isfinite(target)) return set_error(SPAMM_EINVAL, "target must be > 0");
    hipStream_t s = (hipStream_t)stream;
    spamm_status r = ensure_tiers(A, s);
    if (r == SPAMM_OK && B != A) r = ensure_tiers(B, s);
    if (r != SPAMM_OK) return r;
    const int64_t* off = reinterpret_cast<const int64_t*>(A->norms + A->norms_total);
    const int* mm = reinterpret_cast<const int*>(off + kMaxLevels);
    hipLaunchKernelGGL(k_tau_hist, dim3(2 * kTiers), dim3(256), 0, s, A->norms, B->norms, off, mm, A->L, dev_out);
    hipLaunchKernelGGL(k_tau_scalars, dim3(1), dim3(1), 0, s, dev_out, (float)std::log10(target),
                       (float)(std::log2((double)A->nb) / 10.0), (float)(std::log2((double)A->b) / 7.0));
    SPAMM_HIP(hipGetLastError());
    return SPAMM_OK;
}

spamm_status spamm_tau_forward(const spamm_tau_model* m, const float* dev_x, int64_t count, float* dev_y,
                               void* stream) {
    if (!m || !dev_x || !dev_y || count < 1) return set_error(SPAMM_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const Allocator al = current_allocator();
    void* ws = raw_alloc(al, work_bytes(count), s);
    if (!ws) return set_error(SPAMM_ENOMEM, "tau workspace allocation failed");
    const_cast<spamm_tau_model*>(m)->last_stream = s;
    Work w = carve(ws, count);
    w.yhat = dev_y;
    hipError_t e = forward(m->params, dev_x, count, w, s);
    raw_free(al, ws, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "spamm_tau_forward");
    return SPAMM_OK;
}

spamm_status spamm_tau_grad(const spamm_tau_model* m, const float* dev_x, const float* dev_y, int64_t count,
                            float* host_grad, float* host_loss, void* stream) {
    if (!m || !dev_x || !dev_y || count < 1 || !host_grad) return set_error(SPAMM_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const Allocator al = current_allocator();
    void* ws = raw_alloc(al, work_bytes(count), s);
    if (!ws) return set_error(SPAMM_ENOMEM, "tau workspace allocation failed");
    const_cast<spamm_tau_model*>(m)->last_stream = s;
    Work w = carve(ws, count);
    unsigned nb = 0;
    hipError_t e = forward(m->params, dev_x, count, w, s);
    if (e == hipSuccess) e = backward(m->params, dev_x, dev_y, count, w, nb, s);
    std::vector<float> part(8192);
    if (e == hipSuccess) e = hipMemcpyAsync(host_grad, w.grad, (size_t)kNParam * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(part.data(), w.part, (size_t)nb * 4, hipMemcpyDeviceToHost, s);
    raw_free(al, ws, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "spamm_tau_grad");
    if (host_loss) {
        double l = 0.0;
        for (unsigned i = 0; i < nb; ++i) l += part[i];
        *host_loss = (float)(l / (double)count);
    }
    return SPAMM_OK;
}

spamm_status spamm_tau_train(spamm_tau_model* m, const float* dev_x, const float* dev_y, int64_t count, int32_t epochs,
                             int32_t batch, float lr, void* stream, float* host_loss) {
    if (!m || !dev_x || !dev_y || count < 1 || epochs < 1 || batch < 1 || !(lr > 0.0f))
        return set_error(SPAMM_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t B = batch < count ? batch : count;
    const Allocator al = current_allocator();
    void* ws = raw_alloc(al, work_bytes(B), s);
    if (!ws) return set_error(SPAMM_ENOMEM, "tau workspace allocation failed");
    m->last_stream = s;
    Work w = carve(ws, B);
    std::vector<float> part(8192);
    hipError_t e = hipSuccess;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        double loss = 0.0;
        for (int64_t r0 = 0; r0 < count && e == hipSuccess; r0 += B) {
            const int64_t nb = r0 + B <= count ? B : count - r0;
            const float* X = dev_x + r0 * kIn;
            const float* Y = dev_y + r0;
            unsigned lb = 0;
            e = forward(m->params, X, nb, w, s);
            if (e == hipSuccess) e = backward(m->params, X, Y, nb, w, lb, s);
            if (e != hipSuccess) break;
            m->t += 1;
            const float bc1 = 1.0f - std::pow(b1, (float)m->t), bc2 = 1.0f - std::pow(b2, (float)m->t);
            hipLaunchKernelGGL(k_adam, dim3(grid_for(kNParam)), dim3(256), 0, s, m->params, w.grad, m->m, m->v,
                               kNParam, lr, b1, b2, eps, bc1, bc2);
            e = hipGetLastError();
            if (host_loss && e == hipSuccess) {
                e = hipMemcpyAsync(part.data(), w.part, (size_t)lb * 4, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                for (unsigned i = 0; i < lb; ++i) loss += part[i];
            }
        }
        if (host_loss) host_loss[ep] = (float)(loss / (double)count);
    }
    raw_free(al, ws, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "spamm_tau_train");
    return SPAMM_OK;
}

spamm_status spamm_tau_predict(const spamm_matrix* A, const spamm_matrix* B, double target,
                               const spamm_tau_model* m, void* stream, double* tau_out) {
    if (!A || !B || !m || !tau_out) return set_error(SPAMM_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const Allocator al = current_allocator();
    float* buf = (float*)raw_alloc(al, (kIn + 16) * sizeof(float), s);
    if (!buf) return set_error(SPAMM_ENOMEM, "tau workspace allocation failed");
    spamm_status r = spamm_tau_features(A, B, target, buf, stream);
    float yh = 0.0f;
    if (r == SPAMM_OK) r = spamm_tau_forward(m, buf, 1, buf + kIn, stream);
    double ra = 0.0, rb = 0.0;
    hipError_t e = hipSuccess;
    if (r == SPAMM_OK) e = hipMemcpyAsync(&yh, buf + kIn, 4, hipMemcpyDeviceToHost, s);
    if (r == SPAMM_OK && e == hipSuccess) e = hipMemcpyAsync(&ra, A->norms + A->lvl_off[A->L], 8, hipMemcpyDeviceToHost, s);
    if (r == SPAMM_OK && e == hipSuccess) e = hipMemcpyAsync(&rb, B->norms + B->lvl_off[B->L], 8, hipMemcpyDeviceToHost, s);
    raw_free(al, buf, s);
    if (r == SPAMM_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    if (r != SPAMM_OK) return r;
    if (e != hipSuccess) return hip_error(e, "spamm_tau_predict");
    // tau = 10^y ||A||_F ||B||_F
    *tau_out = std::pow(10.0, (double)yh) * std::sqrt(ra) * std::sqrt(rb);
    if (*tau_out > 0.0 && *tau_out < 1e-150) *tau_out = 1e-150;
    return SPAMM_OK;
}

spamm_status spamm_tau_select(const spamm_matrix* A, const spamm_matrix* B, double target, const spamm_tau_model* m,
                              spamm_leaf_prec prec, double resolution_decades, void* stream, spamm_matrix** C,
                              spamm_tau_info* info) {
    if (!A || !B || !C || !info) return set_error(SPAMM_EINVAL, "null argument");
    if (!(target > 0.0)) return set_error(SPAMM_EINVAL, "target must be > 0");
    if (!(resolution_decades > 0.0)) return set_error(SPAMM_EINVAL, "resolution must be > 0");
    std::memset(info, 0, sizeof *info);
    spamm_status r;
    double tau0 = 0.0;
    // the network is asked for half the target so that a typical prediction
    // lands inside it; a miss steps down towards the target (see below)
    const double step = 1.0;
    if (m) {
        if ((r = spamm_tau_predict(A, B, 0.5 * target, m, stream, &tau0)) != SPAMM_OK) return r;
    } else {
        // no model: start one decade above target * ||A||_F ||B||_F
        double ra = 0.0, rb = 0.0;
        if ((r = ensure_tiers(A, (hipStream_t)stream)) != SPAMM_OK) return r;
        if ((r = ensure_tiers(B, (hipStream_t)stream)) != SPAMM_OK) return r;
        SPAMM_HIP(hipStreamSynchronize((hipStream_t)stream));
        SPAMM_HIP(hipMemcpy(&ra, A->norms + A->lvl_off[A->L], 8, hipMemcpyDeviceToHost));
        SPAMM_HIP(hipMemcpy(&rb, B->norms + B->lvl_off[B->L], 8, hipMemcpyDeviceToHost));
        tau0 = 10.0 * target * std::sqrt(ra) * std::sqrt(rb);
    }
    info->tau_pred = tau0;
    // the exact product: FP64 leaves at tau = 0
    spamm_matrix* E = nullptr;
    if ((r = spamm_multiply(A, B, 0.0, SPAMM_LEAF_F64, stream, &E, nullptr)) != SPAMM_OK) return r;
    auto err_at = [&](double tau, double* err, int64_t* tasks) -> spamm_status {
        int64_t t = 0;
        spamm_status q = multiply_count(A, B, tau, prec, (hipStream_t)stream, C, &t);
        if (q != SPAMM_OK) return q;
        double d2 = 0.0, r2 = 0.0;
        if ((q = spamm_diff_norms(*C, E, &d2, &r2, stream)) != SPAMM_OK) return q;
        *err = r2 > 0.0 ? std::sqrt(d2 / r2) : std::sqrt(d2);
        *tasks = t;
        info->evaluations += 1;
        return SPAMM_OK;
    };
    double e0 = 0.0;
    int64_t t0 = 0;
    r = err_at(tau0, &e0, &t0);
    info->err_pred = e0;
    double tau = tau0, err = e0;
    int64_t tasks = t0;
    if (r == SPAMM_OK && e0 > target) {
        info->fallback = 1;
        // step down until the target holds, then bisect in log10(tau) between
        // that tau and the last one that missed.  From a prediction each step
        // aims at the target: the error grows about in proportion to tau (each
        // culled product adds about its norm product), so the step is
        // log10(err / target) plus a tenth of a decade (at least 0.1); with no
        // model the steps are whole decades.
        double hi = std::log10(tau0), lo = hi, elo = e0;
        int64_t tlo = t0;
        bool met = false, last_at_lo = true;
        for (int k = 0; k < 24 && r == SPAMM_OK && lo > std::log10(tau0) - 12.0; ++k) {
            hi = lo;
            lo -= m ? std::max(0.1, std::log10(elo / target) + 0.1) : step;
            r = err_at(std::pow(10.0, lo), &elo, &tlo);
            if (r == SPAMM_OK && elo <= target) {
                met = true;
                break;
            }
        }
        while (r == SPAMM_OK && met && hi - lo > resolution_decades) {
            const double mid = 0.5 * (lo + hi);
            double em = 0.0;
            int64_t tm = 0;
            r = err_at(std::pow(10.0, mid), &em, &tm);
            if (r != SPAMM_OK) break;
            if (em <= target) {
                lo = mid;
                elo = em;
                tlo = tm;
                last_at_lo = true;
            } else {
                hi = mid;
                last_at_lo = false;
            }
        }
        tau = std::pow(10.0, lo);
        err = elo;
        tasks = tlo;
        // leave C holding the product at the returned tau
        if (r == SPAMM_OK && !last_at_lo) r = err_at(tau, &err, &tasks);
    }
    spamm_free(E);
    if (r != SPAMM_OK) return r;
    info->tau = tau;
    info->rel_err = err;
    info->tasks = tasks;
    if (err > target) return set_error(SPAMM_ENOCONV, "no tau met the target within 12 decades");
    return SPAMM_OK;
}

}  // extern "C"
