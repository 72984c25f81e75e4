/*
 * Plain FP64 CPU oracle for Sparse Approximate Matrix Multiplication (SpAMM).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the HIP library is checked against.  Nothing in the product path links,
 * loads or calls it; it shares no code, header or table with the HIP sources.
 *
 * What it computes (Liu et al., "Accelerating Sparse Approximate Matrix
 * Multiplication on GPUs", section 2.1):
 *   - the quadtree split of a matrix into four quadrants per level (Eq. 1);
 *   - the Frobenius norm of every quadtree node (Eq. 2);
 *   - the recursive SpAMM of Algorithm 1: at the lowest level C = A*B; above it,
 *     for every output quadrant (i,j) and k in {0,1}, the sub-product of
 *     A_{i,k} and B_{k,j} is recursed into when ||A_{i,k}||_F*||B_{k,j}||_F >= tau
 *     and replaced by zero otherwise, and C_{i,j} = T0 + T1.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   - The matrix is zero padded to leaf*2^Lv, Lv = ceil(log2(ceil(N/leaf))), so
 *     that the quadtree of Eq. 1 reaches leaf tiles of edge `leaf` (the paper pads
 *     with zeros when the leaf size does not divide N, section 3).
 *   - The root pair is tested too: if ||A||_F*||B||_F < tau the result is zero.
 *     Algorithm 1 only tests children; for N > leaf this changes nothing.
 *   - Norms are FP64: every FP32 input square is exact in FP64, and the sum of
 *     squares uses Neumaier-compensated summation.  Products of node norms are
 *     compared with `>=`, as in Algorithm 1.
 *   - Counted leaf pairs are those with tile indices inside the real
 *     ceil(N/leaf)^3 grid; pairs touching only padding are never counted.
 *
 * Work is split by output leaf tile: the recursion for tile (ti, tj) visits at
 * every level only the output quadrant that contains the tile, which is exactly
 * the part of Algorithm 1 that determines that tile.  Tiles are independent, so
 * they are distributed over OpenMP threads; this changes no arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int64_t oracle_bdim(int64_t n, int32_t leaf) {
    if (n <= 0 || leaf <= 0) return 0;
    return (n + leaf - 1) / leaf;
}

int32_t oracle_levels(int64_t n, int32_t leaf) {
    int64_t b = oracle_bdim(n, leaf);
    int32_t lv = 0;
    while (((int64_t)1 << lv) < b) ++lv;
    return lv;
}

static int64_t level_offset(int32_t l) { return (((int64_t)1 << (2 * l)) - 1) / 3; }

int64_t oracle_pyramid_size(int64_t n, int32_t leaf) {
    return level_offset(oracle_levels(n, leaf) + 1);
}

int32_t oracle_max_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. 2 for one node: sqrt of the sum of squares of the node's elements, taken
 * over the part of the node that lies inside the N x N matrix (the padding is
 * zero).  Neumaier summation in row-major order. */
static double node_norm(const float* x, int64_t n, int64_t r0, int64_t c0, int64_t size) {
    int64_t r1 = r0 + size < n ? r0 + size : n;
    int64_t c1 = c0 + size < n ? c0 + size : n;
    double sum = 0.0, comp = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const float* row = x + r * n;
        for (int64_t c = c0; c < c1; ++c) {
            double v = (double)row[c];
            double t = v * v;
            double y = sum + t;
            if (fabs(sum) >= fabs(t))
                comp += (sum - y) + t;
            else
                comp += (t - y) + sum;
            sum = y;
        }
    }
    return sqrt(sum + comp);
}

/* Frobenius norms of every quadtree node, levels 0 (root) .. Lv (leaf tiles).
 * Level l holds 2^l x 2^l nodes of edge leaf*2^(Lv-l), row-major, at offset
 * (4^l - 1)/3.  Each node is summed directly from the matrix elements, so no
 * level is derived from another. */
int oracle_pyramid(const float* x, int64_t n, int32_t leaf, double* pyr) {
    if (!x || !pyr || n <= 0 || leaf <= 0) return 1;
    int32_t lv = oracle_levels(n, leaf);
    for (int32_t l = 0; l <= lv; ++l) {
        int64_t side = (int64_t)1 << l;
        int64_t size = (int64_t)leaf << (lv - l);
        double* out = pyr + level_offset(l);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t idx = 0; idx < side * side; ++idx) {
            int64_t a = idx / side, b = idx % side;
            out[idx] = node_norm(x, n, a * size, b * size, size);
        }
    }
    return 0;
}

typedef struct {
    const float *a, *b;
    int64_t n, bdim;
    int32_t leaf, lv;
    double tau;
    const double *pa, *pb;
} ctx_t;

static double pnorm(const double* pyr, int32_t l, int64_t r, int64_t c) {
    return pyr[level_offset(l) + r * ((int64_t)1 << l) + c];
}

/* Copy the leaf tile (tr, tc) of x into dst (leaf x leaf, FP64), zero padded. */
static void load_tile(const float* x, int64_t n, int32_t leaf, int64_t tr, int64_t tc, double* dst) {
    for (int32_t r = 0; r < leaf; ++r) {
        int64_t gr = tr * leaf + r;
        for (int32_t c = 0; c < leaf; ++c) {
            int64_t gc = tc * leaf + c;
            dst[(int64_t)r * leaf + c] = (gr < n && gc < n) ? (double)x[gr * n + gc] : 0.0;
        }
    }
}

/* Lowest level of Algorithm 1: out = A[ti,k] * B[k,tj], plain triple loop. */
static void leaf_product(const ctx_t* c, int64_t ti, int64_t k, int64_t tj, double* out, double* ta, double* tb) {
    int32_t L = c->leaf;
    load_tile(c->a, c->n, L, ti, k, ta);
    load_tile(c->b, c->n, L, k, tj, tb);
    memset(out, 0, sizeof(double) * (size_t)L * L);
    for (int32_t r = 0; r < L; ++r)
        for (int32_t q = 0; q < L; ++q) {
            double arq = ta[(int64_t)r * L + q];
            const double* brow = tb + (int64_t)q * L;
            double* orow = out + (int64_t)r * L;
            for (int32_t s = 0; s < L; ++s) orow[s] += arq * brow[s];
        }
}

/* Algorithm 1 applied to the pair (A node (I, K), B node (K, J)) at level l,
 * where (I, J) is the level-l output node containing leaf tile (ti, tj).
 * Writes that tile's part of the result into out (NULL: count only).
 * ops holds 2*leaf^2 doubles for the leaf operands; tstack holds one leaf^2
 * buffer (T1) per remaining level. */
static void rec(const ctx_t* c, int32_t l, int64_t K, int64_t ti, int64_t tj, double* out, double* ops,
                double* tstack, uint8_t* mask_row, int64_t* count) {
    int32_t L = c->leaf;
    int64_t L2 = (int64_t)L * L;
    if (l == c->lv) {
        if (K < c->bdim) {
            if (mask_row) mask_row[K] = 1;
            ++*count;
        }
        if (out) leaf_product(c, ti, K, tj, out, ops, ops + L2);
        return;
    }
    int32_t sh = c->lv - (l + 1);
    int64_t I = ti >> sh, J = tj >> sh;
    double* t0 = out;
    double* t1 = out ? tstack : NULL;
    double* deeper = out ? tstack + L2 : NULL;
    for (int kk = 0; kk < 2; ++kk) {
        int64_t kc = 2 * K + kk;
        double* t = kk == 0 ? t0 : t1;
        if (pnorm(c->pa, l + 1, I, kc) * pnorm(c->pb, l + 1, kc, J) >= c->tau) {
            rec(c, l + 1, kc, ti, tj, t, ops, deeper, mask_row, count);
        } else if (t) {
            memset(t, 0, sizeof(double) * (size_t)L2);
        }
    }
    if (out)
        for (int64_t e = 0; e < L2; ++e) t0[e] = t0[e] + t1[e];
}

/* SpAMM (Algorithm 1, with the root pair tested) for the listed output leaf
 * tiles.  tiles: ntiles pairs (ti, tj), 0 <= ti, tj < bdim.  pyrA/pyrB: node
 * norms from oracle_pyramid.  ctiles: ntiles x leaf x leaf FP64 results, or NULL
 * to only count.  mask: ntiles x bdim bytes, mask[t*bdim + k] = 1 when the leaf
 * pair (ti, k, tj) was multiplied, or NULL.  counts: pairs multiplied per tile.
 * Returns 0, or 1 on bad arguments, 2 on allocation failure. */
int oracle_spamm_tiles(const float* a, const float* b, int64_t n, int32_t leaf, double tau, const double* pyr_a,
                       const double* pyr_b, const int64_t* tiles, int64_t ntiles, double* ctiles, uint8_t* mask,
                       int64_t* counts) {
    if (!a || !b || !pyr_a || !pyr_b || !counts || n <= 0 || leaf <= 0 || ntiles < 0 || (ntiles > 0 && !tiles))
        return 1;
    if (isnan(tau)) return 1;
    ctx_t c;
    c.a = a;
    c.b = b;
    c.n = n;
    c.leaf = leaf;
    c.lv = oracle_levels(n, leaf);
    c.bdim = oracle_bdim(n, leaf);
    c.tau = tau;
    c.pa = pyr_a;
    c.pb = pyr_b;
    for (int64_t t = 0; t < ntiles; ++t)
        if (tiles[2 * t] < 0 || tiles[2 * t] >= c.bdim || tiles[2 * t + 1] < 0 || tiles[2 * t + 1] >= c.bdim)
            return 1;
    int64_t L2 = (int64_t)leaf * leaf;
    int failed = 0;
#pragma omp parallel
    {
        /* leaf operands (2*L2), then one T1 buffer per level */
        double* stack = ctiles ? (double*)malloc(sizeof(double) * (size_t)L2 * (size_t)(c.lv + 2)) : NULL;
        if (ctiles && !stack) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < ntiles; ++t) {
            if (ctiles && !stack) continue;
            int64_t ti = tiles[2 * t], tj = tiles[2 * t + 1];
            double* out = ctiles ? ctiles + t * L2 : NULL;
            uint8_t* mrow = mask ? mask + t * c.bdim : NULL;
            if (mrow) memset(mrow, 0, (size_t)c.bdim);
            int64_t cnt = 0;
            if (pnorm(c.pa, 0, 0, 0) * pnorm(c.pb, 0, 0, 0) >= tau) {
                rec(&c, 0, 0, ti, tj, out, stack, stack ? stack + 2 * L2 : NULL, mrow, &cnt);
            } else if (out) {
                memset(out, 0, sizeof(double) * (size_t)L2);
            }
            counts[t] = cnt;
        }
        free(stack);
    }
    return failed ? 2 : 0;
}
