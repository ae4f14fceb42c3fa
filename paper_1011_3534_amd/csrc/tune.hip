// Autotuner of the batched product: timed trials over leaf size, operand
// staging and leaf schedule on the caller's own operands, with an error check
// against the exact product, and a line-per-key cache file.  Built only on the
// public ABI.
//
// The leaf size changes which products are kept (the cull tests b x b
// blocks), so a candidate qualifies only if every product of the batch stays
// within max_rel_err of the exact product (FP64 leaves at tau = 0).
//
// The cache key describes the batch by buckets rather than by its exact
// sizes, so that batches of the same shape share an answer: the count in
// octaves, the mean n in half-octaves and the kept fraction of the leaf
// triples (sum of T over sum of nb^3 at the first candidate leaf, in octaves),
// with the element type, leaf precision, error target and candidate leaves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "spamm_internal.hpp"

namespace {

// Octave (step 1) or half-octave (step 0.5) bucket of a positive value.
int bucket(double v, double step) { return (int)std::floor(std::log2(v) / step + 0.5); }

std::string cache_key(int32_t count, const int64_t* n, double density, spamm_dtype dt, spamm_leaf_prec prec,
                      const int32_t* leaves, int32_t n_leaves, double max_rel_err) {
    double sumn = 0.0;
    for (int m = 0; m < count; ++m) sumn += (double)n[m];
    std::ostringstream k;
    k << "gfx950|count=2^" << bucket((double)count, 1.0) << "|n=2^" << 0.5 * bucket(sumn / count, 0.5);
    if (density > 0.0)
        k << "|kept=2^" << bucket(density, 1.0);
    else
        k << "|kept=0";
    k << "|dt=" << (int)dt << "|prec=" << (int)prec;
    char buf[64];
    std::snprintf(buf, sizeof buf, "|err=%.1e|leaves=", max_rel_err);
    k << buf;
    for (int i = 0; i < n_leaves; ++i) k << leaves[i] << (i + 1 < n_leaves ? "," : "");
    return k.str();
}

bool cache_lookup(const char* path, const std::string& key, spamm_tune* best, double* ms) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        std::istringstream rest(line.substr(tab + 1));
        int leaf = 0, sched = 0, split = 0;
        double t = 0.0;
        if (rest >> leaf >> sched >> split >> t) {
            std::memset(best, 0, sizeof *best);
            best->leaf = leaf;
            best->schedule = sched;
            best->split = split;
            *ms = t;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const spamm_tune& best, double ms) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << '\t' << best.leaf << ' ' << best.schedule << ' ' << best.split << ' ' << ms << '\n';
}

struct Handles {
    std::vector<spamm_matrix*> h;
    ~Handles() {
        for (auto* x : h) spamm_free(x);
    }
};

struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

extern "C" spamm_status spamm_autotune_batched(int32_t count, const void* const* dev_a, const int64_t* n,
                                               spamm_dtype dt, const double* tau, spamm_leaf_prec prec,
                                               const int32_t* leaves, int32_t n_leaves, double max_rel_err,
                                               int32_t reps, const char* cache_path, void* stream, spamm_tune* best,
                                               spamm_tune_report* report) {
    using spamm::set_error;
    if (count < 1 || count > spamm::kMaxBatch) return set_error(SPAMM_EINVAL, "count outside [1, 128]");
    if (!dev_a || !n || !tau || !leaves || !best) return set_error(SPAMM_EINVAL, "null argument");
    if (n_leaves < 1 || n_leaves > SPAMM_TUNE_MAX_LEAVES) return set_error(SPAMM_EINVAL, "n_leaves outside [1, 3]");
    if (reps < 1) return set_error(SPAMM_EINVAL, "reps < 1");
    if (!(max_rel_err > 0.0)) return set_error(SPAMM_EINVAL, "max_rel_err must be > 0");
    for (int i = 0; i < n_leaves; ++i)
        if (leaves[i] != 32 && leaves[i] != 64 && leaves[i] != 128)
            return set_error(SPAMM_EINVAL, "leaf candidates must be 32, 64 or 128");
    hipStream_t s = (hipStream_t)stream;
    if (report) std::memset(report, 0, sizeof *report);
    spamm_status r;
    // the operands at the first candidate leaf: one product with statistics
    // gives the kept fraction of the cache key, and they form the exact
    // products (FP64 leaves at tau = 0) of the error check
    Handles exa;
    for (int m = 0; m < count; ++m) {
        spamm_matrix* a = nullptr;
        if ((r = spamm_build(dev_a[m], n[m], n[m], dt, leaves[0], stream, &a)) != SPAMM_OK) return r;
        exa.h.push_back(a);
    }
    double density = 0.0;
    {
        Handles c0;
        c0.h.assign(count, nullptr);
        std::vector<spamm_stats> st(count);
        if ((r = spamm_multiply_batched(count, exa.h.data(), exa.h.data(), tau, prec, nullptr, stream, c0.h.data(),
                                        st.data())) != SPAMM_OK)
            return r;
        double kept = 0.0, all = 0.0;
        for (int m = 0; m < count; ++m) {
            kept += (double)st[m].tasks;
            all += (double)st[m].nb * (double)st[m].nb * (double)st[m].nb;
        }
        density = all > 0.0 ? kept / all : 0.0;
    }
    const std::string key = cache_key(count, n, density, dt, prec, leaves, n_leaves, max_rel_err);
    double cached_ms = 0.0;
    if (cache_lookup(cache_path, key, best, &cached_ms)) {
        if (report) {
            report->from_cache = 1;
            report->best_ms = cached_ms;
        }
        return SPAMM_OK;
    }
    Handles ex;
    for (int m = 0; m < count; ++m) {
        spamm_matrix* e = nullptr;
        if ((r = spamm_multiply(exa.h[m], exa.h[m], 0.0, SPAMM_LEAF_F64, stream, &e, nullptr)) != SPAMM_OK) return r;
        ex.h.push_back(e);
    }
    for (auto* a : exa.h) spamm_free(a);
    exa.h.clear();
    // 16-bit leaves of FP32 operands: the operands are also tried with split
    // tiles (spamm_build_ex), which the leaf kernels read without splitting
    const bool split_axis = dt == SPAMM_F32 && (prec == SPAMM_LEAF_BF16 || prec == SPAMM_LEAF_BF16X3 ||
                                                prec == SPAMM_LEAF_F16 || prec == SPAMM_LEAF_F16X3);
    Events ev;
    SPAMM_HIP(hipEventCreate(&ev.e0));
    SPAMM_HIP(hipEventCreate(&ev.e1));
    double best_ms = INFINITY;
    int trials = 0;
    const int scheds[3] = {SPAMM_SCHED_STATIC, SPAMM_SCHED_LPT, SPAMM_SCHED_LIST};
    for (int trial_set = 0; trial_set < n_leaves * (split_axis ? 2 : 1); ++trial_set) {
        const int li = split_axis ? trial_set / 2 : trial_set, sp = split_axis ? trial_set % 2 : 0;
        Handles hA, hC;
        hC.h.assign(count, nullptr);
        for (int m = 0; m < count; ++m) {
            spamm_matrix* a = nullptr;
            r = sp ? spamm_build_ex(dev_a[m], n[m], n[m], dt, leaves[li], prec, stream, &a)
                   : spamm_build(dev_a[m], n[m], n[m], dt, leaves[li], stream, &a);
            if (r != SPAMM_OK) return r;
            hA.h.push_back(a);
        }
        for (int si = 0; si < 3; ++si) {
            spamm_tune t;
            std::memset(&t, 0, sizeof t);
            t.leaf = leaves[li];
            t.schedule = scheds[si];
            t.split = sp;
            // warm-up (also allocates the results)
            if ((r = spamm_multiply_batched(count, hA.h.data(), hA.h.data(), tau, prec, &t, stream, hC.h.data(),
                                            nullptr)) != SPAMM_OK)
                return r;
            std::vector<float> times;
            for (int k = 0; k < reps; ++k) {
                SPAMM_HIP(hipEventRecord(ev.e0, s));
                if ((r = spamm_multiply_batched(count, hA.h.data(), hA.h.data(), tau, prec, &t, stream, hC.h.data(),
                                                nullptr)) != SPAMM_OK)
                    return r;
                SPAMM_HIP(hipEventRecord(ev.e1, s));
                SPAMM_HIP(hipEventSynchronize(ev.e1));
                float ms = 0.f;
                SPAMM_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
                times.push_back(ms);
            }
            std::sort(times.begin(), times.end());
            const double med = times[times.size() / 2];
            double worst = 0.0;
            for (int m = 0; m < count; ++m) {
                double d2 = 0.0, r2 = 0.0;
                if ((r = spamm_diff_norms(hC.h[m], ex.h[m], &d2, &r2, stream)) != SPAMM_OK) return r;
                worst = std::max(worst, r2 > 0.0 ? std::sqrt(d2 / r2) : std::sqrt(d2));
            }
            const bool ok = worst <= max_rel_err;
            if (report && trials < SPAMM_TUNE_MAX_TRIALS) {
                report->leaf[trials] = t.leaf;
                report->schedule[trials] = t.schedule;
                report->split[trials] = t.split;
                report->ms[trials] = med;
                report->max_rel_err[trials] = worst;
                report->qualified[trials] = ok;
            }
            ++trials;
            if (ok && med < best_ms) {
                best_ms = med;
                *best = t;
            }
        }
    }
    if (report) {
        report->trials = trials;
        report->best_ms = best_ms;
    }
    if (!std::isfinite(best_ms)) return set_error(SPAMM_EINVAL, "no candidate met max_rel_err");
    cache_store(cache_path, key, *best, best_ms);
    return SPAMM_OK;
}
