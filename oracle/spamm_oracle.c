/*
 * CPU oracle for the Sparse Approximate Matrix Multiply (SpAMM).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 definition
 * that the GPU library is checked against.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code, header or table with the HIP library.
 *
 * What it computes (Challacombe & Bock, "Fast Multiplication of Matrices with
 * Decay", section 2):
 *   - the quadtree representation of Eq. (1): matrices split recursively into
 *     2x2 blocks down to dense b x b leaves, with a Frobenius norm carried at
 *     every node (the norm choice is stated in section 3);
 *   - the SpAMM recursion of Eq. (4): a block product is dropped when
 *     ||A^k|| ||B^k|| < tau, computed densely at the finest tier, and
 *     otherwise assembled from the 8 sub-products;
 *   - the same result by flat enumeration of leaf triples (I,J,K);
 *   - the culled-norm sums that bound the omitted part of the product
 *     (section 2, Eq. 3: an omitted block product has norm at most
 *     ||A^k|| ||B^k||), over culled leaf triples or over culled octree nodes.
 *
 * Readings fixed here where the paper is silent:
 *   - norms are carried as FP64 *squared* Frobenius norms S and the cull test
 *     is fl(S_A * S_B) < fl(tau*tau) (no square root anywhere), ties kept;
 *   - canonical summation order of a leaf norm: for every column c the sum
 *     s_c = x_{0c}^2 + x_{1c}^2 + ... is taken sequentially over rows with an
 *     explicit fused multiply-add, then columns are combined by the pairwise
 *     tree s_c <- s_c + s_{c+h}, h = b/2, b/4, ..., 1; S = s_0;
 *   - a parent's S is (S_00 + S_01) + (S_10 + S_11), absent children = +0;
 *   - a C tile sums its kept leaf products P = A_IK B_KJ in ascending K, each
 *     P computed afresh with its inner index ascending.
 * Build with -ffp-contract=off so that no other contraction changes rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_LEVELS 40

static int is_pow2(int32_t b) { return b > 0 && (b & (b - 1)) == 0; }

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Canonical squared Frobenius norm of the b x b leaf (I,K) of a row-major
 * n x n matrix; elements outside the matrix are zero padding. */
static double leaf_sqnorm(const double* a, int64_t n, int64_t lda, int32_t b,
                          int64_t I, int64_t K, double* s /* b scratch */) {
    for (int32_t c = 0; c < b; ++c) {
        double acc = 0.0;
        int64_t col = K * b + c;
        for (int32_t r = 0; r < b; ++r) {
            int64_t row = I * b + r;
            double x = (row < n && col < n) ? a[row * lda + col] : 0.0;
            acc = fma(x, x, acc);
        }
        s[c] = acc;
    }
    for (int32_t h = b / 2; h >= 1; h /= 2)
        for (int32_t c = 0; c < h; ++c) s[c] = s[c] + s[c + h];
    return s[0];
}

/* S[I*nb + K] for every leaf of the quadtree (Eq. 1 with b x b leaves). */
int orc_tile_sqnorms(const double* a, int64_t n, int64_t lda, int32_t b, double* S) {
    if (n < 1 || lda < n || !is_pow2(b)) return -1;
    int64_t nb = ceil_div(n, b);
    double* s = (double*)malloc(sizeof(double) * (size_t)b);
    if (!s) return -2;
    for (int64_t I = 0; I < nb; ++I)
        for (int64_t K = 0; K < nb; ++K) S[I * nb + K] = leaf_sqnorm(a, n, lda, b, I, K, s);
    free(s);
    return 0;
}

/* One tier up the quadtree: P is ceil(m/2) x ceil(m/2). */
void orc_norm_parent(const double* S, int64_t m, double* P) {
    int64_t mp = ceil_div(m, 2);
    for (int64_t I = 0; I < mp; ++I)
        for (int64_t K = 0; K < mp; ++K) {
            double c[4];
            for (int q = 0; q < 4; ++q) {
                int64_t i = 2 * I + (q >> 1), k = 2 * K + (q & 1);
                c[q] = (i < m && k < m) ? S[i * m + k] : 0.0;
            }
            P[I * mp + K] = (c[0] + c[1]) + (c[2] + c[3]);
        }
}

/* Number of tiers above the leaves: m_0 = nb, m_{l+1} = ceil(m_l/2), m_L = 1. */
int32_t orc_num_levels(int64_t nb) {
    int32_t L = 0;
    int64_t m = nb;
    while (m > 1) { m = ceil_div(m, 2); ++L; }
    return L;
}

typedef struct {
    int64_t m[ORC_MAX_LEVELS];
    double* S[ORC_MAX_LEVELS];
    int32_t L;
} pyramid;

static int build_pyramid(const double* a, int64_t n, int32_t b, pyramid* p) {
    int64_t nb = ceil_div(n, b);
    p->L = orc_num_levels(nb);
    if (p->L + 1 > ORC_MAX_LEVELS) return -1;
    int64_t m = nb;
    for (int32_t l = 0; l <= p->L; ++l) {
        p->m[l] = m;
        p->S[l] = (double*)malloc(sizeof(double) * (size_t)(m * m));
        if (!p->S[l]) return -2;
        if (l == 0) orc_tile_sqnorms(a, n, n, b, p->S[0]);
        else orc_norm_parent(p->S[l - 1], p->m[l - 1], p->S[l]);
        m = ceil_div(m, 2);
    }
    return 0;
}

static void free_pyramid(pyramid* p) {
    for (int32_t l = 0; l <= p->L; ++l) free(p->S[l]);
}

/* C_IJ += A_IK * B_KJ on the real (unpadded) index ranges, the product
 * formed afresh in P with ascending inner index, then added to C. */
static void leaf_product_add(const double* a, const double* bm, int64_t n, int32_t b,
                             int64_t I, int64_t J, int64_t K, double* c, double* P) {
    int64_t i0 = I * b, j0 = J * b, k0 = K * b;
    int64_t ni = (n - i0 < b) ? n - i0 : b;
    int64_t nj = (n - j0 < b) ? n - j0 : b;
    int64_t nk = (n - k0 < b) ? n - k0 : b;
    for (int64_t i = 0; i < ni; ++i) {
        double* prow = P + i * b;
        for (int64_t j = 0; j < nj; ++j) prow[j] = 0.0;
        for (int64_t k = 0; k < nk; ++k) {
            double aik = a[(i0 + i) * n + (k0 + k)];
            const double* brow = bm + (k0 + k) * n + j0;
            for (int64_t j = 0; j < nj; ++j) prow[j] = prow[j] + aik * brow[j];
        }
        double* crow = c + (i0 + i) * n + j0;
        for (int64_t j = 0; j < nj; ++j) crow[j] = crow[j] + prow[j];
    }
}

static uint64_t pack_key(int64_t I, int64_t J, int64_t K) {
    return ((uint64_t)I << 42) | ((uint64_t)J << 21) | (uint64_t)K;
}

typedef struct {
    const double *a, *bm;
    int64_t n;
    int32_t b;
    int32_t depth_scaled;  /* 1: tau_{k+1} = tau_k / 8 below the root (section 2) */
    const pyramid *pa, *pb;
    double* c;
    double* P;
    uint64_t* keys;
    int64_t cap, count;
    int64_t* level_kept;
} rec_ctx;

/* Eq. (4), literally: test the pair against the threshold tau of its depth,
 * multiply densely at the finest tier, otherwise recurse into the 8
 * sub-products (k2 innermost, so every C tile receives its contributions in
 * ascending K).  With the depth-scaled schedule the sub-products are tested
 * against tau / 8 (the rigorous variant of section 2); otherwise tau stays. */
static void spamm_rec(rec_ctx* x, int32_t l, int64_t I, int64_t J, int64_t K, double tau) {
    double sa = x->pa->S[l][I * x->pa->m[l] + K];
    double sb = x->pb->S[l][K * x->pb->m[l] + J];
    if (sa * sb < tau * tau) return;
    if (x->level_kept) x->level_kept[l] += 1;
    if (l == 0) {
        leaf_product_add(x->a, x->bm, x->n, x->b, I, J, K, x->c, x->P);
        if (x->keys && x->count < x->cap) x->keys[x->count] = pack_key(I, J, K);
        x->count += 1;
        return;
    }
    int64_t mc = x->pa->m[l - 1];
    double tau_child = x->depth_scaled ? tau / 8.0 : tau;
    for (int i2 = 0; i2 < 2; ++i2)
        for (int j2 = 0; j2 < 2; ++j2)
            for (int k2 = 0; k2 < 2; ++k2) {
                int64_t Ic = 2 * I + i2, Jc = 2 * J + j2, Kc = 2 * K + k2;
                if (Ic < mc && Jc < mc && Kc < mc) spamm_rec(x, l - 1, Ic, Jc, Kc, tau_child);
            }
}

/* Recursive SpAMM of dense row-major FP64 n x n inputs; writes all of C.
 * keys (optional) receives the leaf triples in visit order; level_kept
 * (optional, L+1 entries) counts the kept nodes per tier (0 = leaf).
 * Returns the number of leaf products, or a negative error. */
int64_t orc_spamm_recursive(const double* a, const double* bm, int64_t n, int32_t b, double tau,
                            int32_t depth_scaled, double* c, uint64_t* keys, int64_t keys_cap,
                            int64_t* level_kept) {
    if (n < 1 || !is_pow2(b) || !(tau >= 0.0) || isinf(tau)) return -1;
    pyramid pa, pb;
    memset(&pa, 0, sizeof pa);
    memset(&pb, 0, sizeof pb);
    if (build_pyramid(a, n, b, &pa) || build_pyramid(bm, n, b, &pb)) {
        free_pyramid(&pa);
        free_pyramid(&pb);
        return -2;
    }
    memset(c, 0, sizeof(double) * (size_t)(n * n));
    rec_ctx x = {a, bm, n, b, depth_scaled, &pa, &pb, c, NULL, keys, keys_cap, 0, level_kept};
    x.P = (double*)malloc(sizeof(double) * (size_t)b * (size_t)b);
    if (level_kept) memset(level_kept, 0, sizeof(int64_t) * (size_t)(pa.L + 1));
    spamm_rec(&x, pa.L, 0, 0, 0, tau);
    free(x.P);
    free_pyramid(&pa);
    free_pyramid(&pb);
    return x.count;
}

/* Flat SpAMM over the C tile rows [I0, I1): keep(I,J,K) <=> !(S_A[I,K] S_B[K,J] < tau^2)
 * on the leaf norms; every C tile sums its kept products in ascending K.
 * Rows of C outside [I0*b, I1*b) are left untouched.  sym_upper (the
 * symmetric squaring of a symmetric A = B, all rows): only the tiles with
 * I <= J are formed by the rule, and C_JI is set to the transpose of C_IJ.
 * Returns the number of leaf products taken. */
int64_t orc_spamm_flat(const double* a, const double* bm, int64_t n, int32_t b, double tau,
                       int64_t I0, int64_t I1, int32_t sym_upper, double* c) {
    if (n < 1 || !is_pow2(b) || !(tau >= 0.0) || isinf(tau)) return -1;
    int64_t nb = ceil_div(n, b);
    if (I0 < 0 || I1 > nb || I0 > I1) return -1;
    if (sym_upper && (I0 != 0 || I1 != nb)) return -1;
    double* SA = (double*)malloc(sizeof(double) * (size_t)(nb * nb));
    double* SB = (double*)malloc(sizeof(double) * (size_t)(nb * nb));
    orc_tile_sqnorms(a, n, n, b, SA);
    orc_tile_sqnorms(bm, n, n, b, SB);
    double tau2 = tau * tau;
    for (int64_t i = I0 * b; i < n && i < I1 * b; ++i) memset(c + i * n, 0, sizeof(double) * (size_t)n);
    int64_t total = 0;
    int64_t ntiles = (I1 - I0) * nb;
#pragma omp parallel reduction(+ : total)
    {
        double* P = (double*)malloc(sizeof(double) * (size_t)b * (size_t)b);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < ntiles; ++t) {
            int64_t I = I0 + t / nb, J = t % nb;
            if (sym_upper && J < I) continue;
            for (int64_t K = 0; K < nb; ++K) {
                if (SA[I * nb + K] * SB[K * nb + J] < tau2) continue;
                leaf_product_add(a, bm, n, b, I, J, K, c, P);
                total += 1;
            }
        }
        free(P);
    }
    if (sym_upper)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                if (j / b < i / b) c[i * n + j] = c[j * n + i];
    free(SA);
    free(SB);
    return total;
}

/* Brute-force enumeration of the kept leaf triples from given leaf norms
 * (nb x nb row-major each).  Keys are written in (I, J, K) lexicographic order
 * (up to cap); culled_bound (optional) receives the sum over culled triples
 * of sqrt(S_A) sqrt(S_B), the Eq. (3) bound on the omitted product.  Returns
 * the number of kept triples. */
int64_t orc_tasks_flat(const double* SA, const double* SB, int64_t nb, double tau,
                       uint64_t* keys, int64_t cap, double* culled_bound) {
    double tau2 = tau * tau;
    int64_t count = 0;
    double bound = 0.0;
    for (int64_t I = 0; I < nb; ++I)
        for (int64_t J = 0; J < nb; ++J)
            for (int64_t K = 0; K < nb; ++K) {
                double sa = SA[I * nb + K], sb = SB[K * nb + J];
                if (sa * sb < tau2) {
                    bound += sqrt(sa) * sqrt(sb);
                    continue;
                }
                if (keys && count < cap) keys[count] = pack_key(I, J, K);
                ++count;
            }
    if (culled_bound) *culled_bound = bound;
    return count;
}

/* The hierarchical test alone (no products): the product-space octree nodes
 * that pass at every tier, with the threshold schedule of spamm_rec.
 * level_kept has L+1 entries; keys (optional) receives the kept leaf triples
 * in visit order.  Returns the leaf count. */
typedef struct {
    const pyramid *pa, *pb;
    int32_t depth_scaled;
    int64_t* level_kept;
    uint64_t* keys;
    int64_t cap, count;
    double bound;  /* sum over culled nodes of sqrt(S_A) sqrt(S_B) */
} count_ctx;

static void count_rec(count_ctx* x, int32_t l, int64_t I, int64_t J, int64_t K, double tau) {
    double sa = x->pa->S[l][I * x->pa->m[l] + K];
    double sb = x->pb->S[l][K * x->pb->m[l] + J];
    if (sa * sb < tau * tau) {
        /* Eq. (3): the whole block product under a culled node has norm at
         * most ||A^k||_F ||B^k||_F */
        x->bound += sqrt(sa) * sqrt(sb);
        return;
    }
    x->level_kept[l] += 1;
    if (l == 0) {
        if (x->keys && x->count < x->cap) x->keys[x->count] = pack_key(I, J, K);
        x->count += 1;
        return;
    }
    int64_t mc = x->pa->m[l - 1];
    double tau_child = x->depth_scaled ? tau / 8.0 : tau;
    for (int i2 = 0; i2 < 2; ++i2)
        for (int j2 = 0; j2 < 2; ++j2)
            for (int k2 = 0; k2 < 2; ++k2) {
                int64_t Ic = 2 * I + i2, Jc = 2 * J + j2, Kc = 2 * K + k2;
                if (Ic < mc && Jc < mc && Kc < mc) count_rec(x, l - 1, Ic, Jc, Kc, tau_child);
            }
}

/* Hierarchical kept leaf triples from leaf norms only (the recursion of
 * Eq. 4 with the products left out).  level_kept: L+1 entries, tier 0 =
 * leaves; keys optional (up to cap); culled_bound (optional) receives the
 * sum over the culled octree nodes -- the nodes the recursion tests and
 * drops, at whatever tier -- of sqrt(S_A) sqrt(S_B), which bounds the
 * Frobenius norm of the omitted part of the product (Eq. 3). */
int64_t orc_tasks_hierarchical(const double* SA, const double* SB, int64_t nb, double tau,
                               int32_t depth_scaled, uint64_t* keys, int64_t cap, int64_t* level_kept,
                               double* culled_bound) {
    pyramid pa, pb;
    memset(&pa, 0, sizeof pa);
    memset(&pb, 0, sizeof pb);
    pa.L = pb.L = orc_num_levels(nb);
    int64_t m = nb;
    for (int32_t l = 0; l <= pa.L; ++l) {
        pa.m[l] = pb.m[l] = m;
        pa.S[l] = (double*)malloc(sizeof(double) * (size_t)(m * m));
        pb.S[l] = (double*)malloc(sizeof(double) * (size_t)(m * m));
        if (l == 0) {
            memcpy(pa.S[0], SA, sizeof(double) * (size_t)(m * m));
            memcpy(pb.S[0], SB, sizeof(double) * (size_t)(m * m));
        } else {
            orc_norm_parent(pa.S[l - 1], pa.m[l - 1], pa.S[l]);
            orc_norm_parent(pb.S[l - 1], pb.m[l - 1], pb.S[l]);
        }
        m = ceil_div(m, 2);
    }
    memset(level_kept, 0, sizeof(int64_t) * (size_t)(pa.L + 1));
    count_ctx x = {&pa, &pb, depth_scaled, level_kept, keys, cap, 0, 0.0};
    count_rec(&x, pa.L, 0, 0, 0, tau);
    if (culled_bound) *culled_bound = x.bound;
    free_pyramid(&pa);
    free_pyramid(&pb);
    return x.count;
}
