/*
 * oracle.c -- plain CPU oracle for the multiple-random-projection-tree (MRPT)
 * voting search of "Fast k-NN Search" (Hyvonen et al., arXiv:1509.06957).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU query path computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU library and never includes or
 * links it; the product path must never call it.
 *
 * Every function follows one passage of the paper:
 *   - random matrix           : Sec. II-B (sparse Gaussian entries), Alg. 1
 *   - projection P = X R      : Sec. II-C, Alg. 1 (projection step), Alg. 3
 *   - grow_tree               : Sec. II-A (median split, left child gets
 *                               ceil(m/2) points), Alg. 2
 *   - tree_query (routing)    : Sec. III (q^T r <= s goes left), Alg. 3
 *   - voting                  : Sec. III-A (f_t, F, S = {F >= v}), Alg. 4
 *   - knn / brute force       : Sec. I-A (k-NN definition, Euclidean metric)
 *   - precision arms          : not in the paper.  bfloat16 and fp8 (OCP
 *                               E4M3, per-row scale) copies of the rows, a
 *                               ranking of S by the distance to the decoded
 *                               row, the best kp kept, and the exact k-NN
 *                               (Sec. I-A) of those kept
 *
 * Readings taken where the paper is silent (listed in the design notes):
 *   - the generator is Philox4x64-10 (Salmon et al., SC'11) keyed by
 *     (seed, 0) with counter (i, level, tree, 0); word 0 decides the
 *     Bernoulli(a) draw, words 1 and 2 feed a Box-Muller normal in double;
 *   - exact-count mode (footnote of Sec. II-D): the ceil(a d) features with
 *     the smallest word-0 uniforms (ties by feature) are the nonzeros;
 *   - projections are float32, one fused multiply-add per nonzero in
 *     ascending feature order starting from +0;
 *   - ties in a node are broken by point id (sort key (projection, id)); the
 *     first ceil(m/2) go left; the stored split is the middle value for odd m
 *     and the float32 midpoint of the two middle values for even m;
 *   - distances are computed in float64; k-NN order is (distance, id);
 *   - bfloat16 rounds to nearest, ties to even; fp8 rows carry the scale
 *     max|x| / 240 (float32), each value x / scale (float32 division) rounded
 *     to the nearest E4M3 value, ties to the even code; the prefilter score
 *     of x is the squared float64 distance between q and the decoded row.
 *
 * Compile: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11.  Round function: two 64x64->128 products, the    */
/* high halves xor-ed with the other counter words and the key; the key is    */
/* bumped by the Weyl constants between rounds.                               */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        __uint128_t p0 = (__uint128_t)PHILOX_M0 * c0;
        __uint128_t p1 = (__uint128_t)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Sparse random matrix, Sec. II-B / Alg. 1: entry (i, level) of tree t is    */
/* N(0,1) with probability a and 0 otherwise.  Stored dense here, row         */
/* (t*depth + level) of length d.  a is compared in double.                   */
/* ------------------------------------------------------------------------ */
void oracle_random_matrix(int32_t d, int32_t T, int32_t depth, float a, uint64_t seed, float *R)
{
    const double two_pow_m53 = 1.0 / 9007199254740992.0;
    const uint64_t key[2] = {seed, 0};
    for (int32_t t = 0; t < T; t++)
        for (int32_t lv = 0; lv < depth; lv++)
            for (int32_t i = 0; i < d; i++) {
                uint64_t ctr[4] = {(uint64_t)i, (uint64_t)lv, (uint64_t)t, 0};
                uint64_t w[4];
                oracle_philox4x64_10(ctr, key, w);
                double u = (double)(w[0] >> 11) * two_pow_m53;          /* [0,1)  */
                float r = 0.0f;
                if (u < (double)a) {
                    double u1 = (double)((w[1] >> 11) + 1) * two_pow_m53; /* (0,1]  */
                    double u2 = (double)(w[2] >> 11) * two_pow_m53;       /* [0,1)  */
                    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                    r = (float)z;
                }
                R[((int64_t)t * depth + lv) * d + i] = r;
            }
}

/* ------------------------------------------------------------------------ */
/* Exact-count variant (the footnote of Sec. II-D): every vector has exactly   */
/* m = ceil(a d) nonzero entries instead of a Bernoulli(a) count.  Reading:    */
/* the m features with the smallest selection uniforms u_i (word 0 of entry    */
/* i's block, ties by i) carry their entry's normal (words 1 and 2), so a      */
/* uniformly random m-subset of the features.  With a = 1 it is the Bernoulli */
/* form (every u_i < 1).  m is ceil of a*d in double, clamped to [1, d].      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double u;
    int32_t i;
} oracle_sel_key;

static int oracle_sel_cmp(const void *x, const void *y)
{
    const oracle_sel_key *p = (const oracle_sel_key *)x, *q = (const oracle_sel_key *)y;
    if (p->u < q->u) return -1;
    if (p->u > q->u) return 1;
    return (p->i > q->i) - (p->i < q->i);
}

int32_t oracle_exact_nnz(int32_t d, float a)
{
    double m = ceil((double)a * (double)d);
    if (m < 1.0) m = 1.0;
    if (m > (double)d) m = (double)d;
    return (int32_t)m;
}

void oracle_random_matrix_exact(int32_t d, int32_t T, int32_t depth, float a, uint64_t seed, float *R)
{
    const double two_pow_m53 = 1.0 / 9007199254740992.0;
    const uint64_t key[2] = {seed, 0};
    const int32_t m = oracle_exact_nnz(d, a);
    oracle_sel_key *keys = (oracle_sel_key *)malloc(sizeof(oracle_sel_key) * (size_t)d);
    for (int32_t t = 0; t < T; t++)
        for (int32_t lv = 0; lv < depth; lv++) {
            float *row = R + ((int64_t)t * depth + lv) * d;
            for (int32_t i = 0; i < d; i++) {
                uint64_t ctr[4] = {(uint64_t)i, (uint64_t)lv, (uint64_t)t, 0};
                uint64_t w[4];
                oracle_philox4x64_10(ctr, key, w);
                keys[i].u = (double)(w[0] >> 11) * two_pow_m53;
                keys[i].i = i;
                row[i] = 0.0f;
            }
            qsort(keys, (size_t)d, sizeof(oracle_sel_key), oracle_sel_cmp);
            for (int32_t r = 0; r < m; r++) {
                const int32_t i = keys[r].i;
                uint64_t ctr[4] = {(uint64_t)i, (uint64_t)lv, (uint64_t)t, 0};
                uint64_t w[4];
                oracle_philox4x64_10(ctr, key, w);
                double u1 = (double)((w[1] >> 11) + 1) * two_pow_m53; /* (0,1]  */
                double u2 = (double)(w[2] >> 11) * two_pow_m53;       /* [0,1)  */
                row[i] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
            }
        }
    free(keys);
}

/* ------------------------------------------------------------------------ */
/* Projection (Sec. II-C, Alg. 1 and Alg. 3): P[x, row] = sum_i X[x,i] R[row,i] */
/* as a float32 chain of fused multiply-adds over the nonzero entries of the  */
/* row in ascending i, starting from +0.                                      */
/* ------------------------------------------------------------------------ */
static float project_one(const float *x, const float *rrow, int32_t d)
{
    float acc = 0.0f;
    for (int32_t i = 0; i < d; i++)
        if (rrow[i] != 0.0f)
            acc = fmaf(x[i], rrow[i], acc);
    return acc;
}

void oracle_project(const float *X, int64_t n, int32_t d, const float *R, int32_t rows, float *P)
{
    for (int64_t x = 0; x < n; x++)
        for (int32_t r = 0; r < rows; r++)
            P[x * rows + r] = project_one(X + x * d, R + (int64_t)r * d, d);
}

/* number of points in every leaf follows from (n, depth) alone: a node with m */
/* points sends ceil(m/2) left and floor(m/2) right (Sec. II-A).  off[L] is    */
/* the first slot of leaf L (leaves in left-to-right order).                   */
static void leaf_sizes_rec(int64_t m, int32_t level, int32_t depth, int64_t node, int64_t *sizes)
{
    if (level == depth) {
        sizes[node - (((int64_t)1 << depth) - 1)] = m;
        return;
    }
    leaf_sizes_rec((m + 1) / 2, level + 1, depth, 2 * node + 1, sizes);
    leaf_sizes_rec(m / 2, level + 1, depth, 2 * node + 2, sizes);
}

void oracle_leaf_offsets(int64_t n, int32_t depth, int64_t *off)
{
    int64_t nleaf = (int64_t)1 << depth;
    int64_t *sizes = (int64_t *)malloc(sizeof(int64_t) * nleaf);
    leaf_sizes_rec(n, 0, depth, 0, sizes);
    off[0] = 0;
    for (int64_t L = 0; L < nleaf; L++)
        off[L + 1] = off[L] + sizes[L];
    free(sizes);
}

/* ------------------------------------------------------------------------ */
/* grow_tree (Alg. 2) with the median split of Sec. II-A.                      */
/* ------------------------------------------------------------------------ */
typedef struct { float val; int32_t id; } keyed_t;

static int cmp_keyed(const void *pa, const void *pb)
{
    const keyed_t *a = (const keyed_t *)pa, *b = (const keyed_t *)pb;
    if (a->val < b->val) return -1;
    if (a->val > b->val) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

static int cmp_id(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

typedef struct {
    const float *P;     /* n x depth projections of this tree */
    int32_t depth;
    float *splits;      /* 2^depth - 1, heap order */
    int32_t *perm;      /* n ids, leaf after leaf */
    int64_t cursor;     /* next free slot in perm */
    keyed_t *keys;      /* scratch */
} grow_ctx;

static void grow_tree(grow_ctx *c, int32_t *ids, int64_t m, int32_t level, int64_t node)
{
    if (level == c->depth) {                       /* leaf: store its point ids */
        qsort(ids, (size_t)m, sizeof(int32_t), cmp_id);
        memcpy(c->perm + c->cursor, ids, sizeof(int32_t) * (size_t)m);
        c->cursor += m;
        return;
    }
    for (int64_t i = 0; i < m; i++) {
        float p = c->P[(int64_t)ids[i] * c->depth + level];
        if (p == 0.0f) p = 0.0f;                   /* -0 and +0 are one value */
        c->keys[i].val = p;
        c->keys[i].id = ids[i];
    }
    qsort(c->keys, (size_t)m, sizeof(keyed_t), cmp_keyed);
    for (int64_t i = 0; i < m; i++)
        ids[i] = c->keys[i].id;
    int64_t nl = (m + 1) / 2;                      /* ceil(m/2) points go left */
    float split;
    if (m % 2 == 1) {
        split = c->keys[nl - 1].val;
    } else {
        float s = c->keys[nl - 1].val + c->keys[nl].val;
        split = s * 0.5f;
    }
    c->splits[node] = split;
    grow_tree(c, ids, nl, level + 1, 2 * node + 1);
    grow_tree(c, ids + nl, m - nl, level + 1, 2 * node + 2);
}

/* Build one tree t: P = X R_t (Alg. 1), then grow_tree from the root. */
static void build_one_tree(const float *X, int64_t n, int32_t d, int32_t depth,
                           const float *Rt, float *splits, int32_t *perm)
{
    float *P = (float *)malloc(sizeof(float) * (size_t)(n * (depth > 0 ? depth : 1)));
    if (depth > 0)
        oracle_project(X, n, d, Rt, depth, P);
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) ids[i] = (int32_t)i;
    grow_ctx c;
    c.P = P; c.depth = depth; c.splits = splits; c.perm = perm; c.cursor = 0;
    c.keys = (keyed_t *)malloc(sizeof(keyed_t) * (size_t)n);
    grow_tree(&c, ids, n, 0, 0);
    free(c.keys); free(ids); free(P);
}

typedef struct {
    const float *X; int64_t n; int32_t d; int32_t T; int32_t depth;
    const float *R; float *splits; int32_t *perm;
    int32_t first, stride;
} build_job;

static void *build_worker(void *arg)
{
    build_job *j = (build_job *)arg;
    int64_t nsplit = ((int64_t)1 << j->depth) - 1;
    for (int32_t t = j->first; t < j->T; t += j->stride)
        build_one_tree(j->X, j->n, j->d, j->depth, j->R + (int64_t)t * j->depth * j->d,
                       j->splits + (int64_t)t * nsplit, j->perm + (int64_t)t * j->n);
    return NULL;
}

/* grow_trees (Alg. 1).  R_out: (T*depth) x d dense; splits: T x (2^depth-1);
 * perm: T x n.  Trees are independent, so they are spread over threads. */
void oracle_build(const float *X, int64_t n, int32_t d, int32_t T, int32_t depth, float a,
                  uint64_t seed, int32_t exact_nnz, float *R_out, float *splits, int32_t *perm,
                  int32_t nthreads)
{
    if (exact_nnz) oracle_random_matrix_exact(d, T, depth, a, seed, R_out);
    else oracle_random_matrix(d, T, depth, a, seed, R_out);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > T) nthreads = T;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    build_job *jobs = (build_job *)malloc(sizeof(build_job) * (size_t)nthreads);
    for (int32_t w = 0; w < nthreads; w++) {
        build_job j = {X, n, d, T, depth, R_out, splits, perm, w, nthreads};
        jobs[w] = j;
        pthread_create(&th[w], NULL, build_worker, &jobs[w]);
    }
    for (int32_t w = 0; w < nthreads; w++) pthread_join(th[w], NULL);
    free(jobs); free(th);
}

/* ------------------------------------------------------------------------ */
/* tree_query (Alg. 3): project q onto the tree's level vectors and descend:  */
/* left when the projection is <= the node's split.  Returns the leaf index.  */
/* ------------------------------------------------------------------------ */
static int32_t route_one(const float *q, int32_t d, const float *Rt, int32_t depth, const float *splits)
{
    int64_t node = 0;
    for (int32_t lv = 0; lv < depth; lv++) {
        float p = project_one(q, Rt + (int64_t)lv * d, d);
        if (p <= splits[node]) node = 2 * node + 1;
        else node = 2 * node + 2;
    }
    return (int32_t)(node - (((int64_t)1 << depth) - 1));
}

void oracle_route(const float *Q, int64_t nq, int32_t d, const float *R, int32_t T, int32_t depth,
                  const float *splits, int32_t *leaf)
{
    int64_t nsplit = ((int64_t)1 << depth) - 1;
    for (int64_t q = 0; q < nq; q++)
        for (int32_t t = 0; t < T; t++)
            leaf[q * T + t] = route_one(Q + q * d, d, R + (int64_t)t * depth * d, depth,
                                        splits + (int64_t)t * nsplit);
}

/* ------------------------------------------------------------------------ */
/* Exact distance (Sec. I-A), float64 throughout.                              */
/* ------------------------------------------------------------------------ */
double oracle_distance(const float *q, const float *x, int32_t d)
{
    double s = 0.0;
    for (int32_t i = 0; i < d; i++) {
        double diff = (double)q[i] - (double)x[i];
        s += diff * diff;
    }
    return sqrt(s);
}

typedef struct { double dist; int32_t id; } cand_t;

static int cmp_cand(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->dist < b->dist) return -1;
    if (a->dist > b->dist) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* knn(q, k, S): exact search restricted to S; order (distance, id); short
 * answers are padded with id -1 and distance +inf. */
static void knn_in_set(const float *q, const float *X, int32_t d, const int32_t *S, int64_t ns,
                       int32_t k, cand_t *scratch, int32_t *out_idx, double *out_dist)
{
    for (int64_t s = 0; s < ns; s++) {
        scratch[s].id = S[s];
        scratch[s].dist = oracle_distance(q, X + (int64_t)S[s] * d, d);
    }
    qsort(scratch, (size_t)ns, sizeof(cand_t), cmp_cand);
    for (int32_t r = 0; r < k; r++) {
        if (r < ns) { out_idx[r] = scratch[r].id; out_dist[r] = scratch[r].dist; }
        else        { out_idx[r] = -1;            out_dist[r] = INFINITY; }
    }
}

/* ------------------------------------------------------------------------ */
/* Low-precision copies of the rows for the prefilter arms.  These are not in */
/* the paper: the arms rank S by an approximate distance, then take the exact */
/* k-NN of the best kp (the stated readings are listed in the design notes).  */
/* ------------------------------------------------------------------------ */

/* bfloat16: the float32 value rounded to 8 significant bits (7 stored), */
/* round to nearest, ties to the even significand.  Written from the       */
/* definition: the two neighbouring bfloat16 values of x are found (toward  */
/* zero: x with its 16 low bits cleared; away from zero: the next one), and */
/* the nearer is taken; a tie goes to the one whose last stored bit is 0.   */
double oracle_bf16_value(uint16_t b)
{
    uint32_t w = (uint32_t)b << 16;
    float f;
    memcpy(&f, &w, sizeof(f));
    return (double)f;
}

uint16_t oracle_bf16_round(float x)
{
    uint32_t w;
    memcpy(&w, &x, sizeof(w));
    uint16_t lo = (uint16_t)(w >> 16);                  /* toward zero */
    if ((w & 0xffffu) == 0u) return lo;                 /* representable */
    if (((lo >> 7) & 0xffu) == 0xffu) return lo;        /* NaN stays NaN */
    uint16_t hi = (uint16_t)(lo + 1u);                  /* next magnitude up */
    double dx = fabs((double)x);
    double dlo = dx - fabs(oracle_bf16_value(lo));
    double dhi = fabs(oracle_bf16_value(hi)) - dx;      /* +inf beyond the largest value */
    if (dlo < dhi) return lo;
    if (dhi < dlo) return hi;
    return (lo & 1u) ? hi : lo;                         /* tie: even significand */
}

void oracle_to_bf16(const float *x, int64_t count, uint16_t *out)
{
    for (int64_t i = 0; i < count; i++) out[i] = oracle_bf16_round(x[i]);
}

/* FP8 E4M3 in the OCP 8-bit floating-point format ("E4M3FN"): 1 sign bit,   */
/* 4 exponent bits with bias 7, 3 significand bits; exponent field 0 holds   */
/* the subnormals m/8 * 2^-6; exponent field 15 with significand 7 is NaN   */
/* (no infinities), so the largest finite value is 1.75 * 2^8 = 448.         */
double oracle_e4m3_value(uint8_t code)
{
    int sign = (code >> 7) & 1;
    int e = (code >> 3) & 15;
    int m = code & 7;
    double mag;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) mag = ldexp((double)m / 8.0, -6);
    else mag = ldexp(1.0 + (double)m / 8.0, e - 7);
    return sign ? -mag : mag;
}

/* round to nearest, ties to the even code, for finite |y| <= 448 (beyond */
/* that the code is NaN); the sign of y is kept (a negative value that    */
/* rounds to zero gives -0).  The non-negative finite codes 0x00 .. 0x7e   */
/* decode to increasing values, so the two codes around |y| are found by  */
/* bisection and the nearer one is taken.                                  */
uint8_t oracle_e4m3_round(float y)
{
    double a = fabs((double)y);
    uint8_t sign = signbit(y) ? 0x80u : 0u;
    if (!(a <= 448.0)) return (uint8_t)(sign | 0x7fu);
    int lo = 0, hi = 0x7e;                              /* value(lo) <= a <= value(hi) */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (oracle_e4m3_value((uint8_t)mid) <= a) lo = mid;
        else hi = mid;
    }
    double dlo = a - oracle_e4m3_value((uint8_t)lo);
    double dhi = oracle_e4m3_value((uint8_t)hi) - a;
    int best;
    if (dlo < dhi) best = lo;
    else if (dhi < dlo) best = hi;
    else best = (lo % 2 == 0) ? lo : hi;                /* tie: the even code */
    return (uint8_t)(sign | (uint8_t)best);
}

/* Per-row scaled fp8 rows: scale = max_i |x_i| / 240 in float32 (1 for an */
/* all-zero row), code_i = e4m3(x_i / scale) with the division in float32,  */
/* decoded value scale * e4m3value(code_i); norm = sum of the decoded       */
/* values squared, in float64.                                              */
static float fp8_row(const float *x, int32_t d, uint8_t *codes, double *decoded)
{
    float mx = 0.0f;
    for (int32_t i = 0; i < d; i++) {
        float ax = fabsf(x[i]);
        if (ax > mx) mx = ax;
    }
    float s = mx > 0.0f ? mx / 240.0f : 1.0f;
    for (int32_t i = 0; i < d; i++) {
        uint8_t c = oracle_e4m3_round(x[i] / s);
        if (codes) codes[i] = c;
        if (decoded) decoded[i] = (double)s * oracle_e4m3_value(c);
    }
    return s;
}

void oracle_to_fp8_rows(const float *X, int64_t n, int32_t d, uint8_t *codes, float *scale, double *norm)
{
    double *dec = (double *)malloc(sizeof(double) * (size_t)d);
    for (int64_t r = 0; r < n; r++) {
        scale[r] = fp8_row(X + r * d, d, codes + r * d, dec);
        double nn = 0.0;
        for (int32_t i = 0; i < d; i++) nn += dec[i] * dec[i];
        norm[r] = nn;
    }
    free(dec);
}

/* the decoded low-precision copy of one row: arm 1 bfloat16, arm 2 fp8 */
static void decode_row(int32_t arm, const float *x, int32_t d, double *out)
{
    if (arm == 1) {
        for (int32_t i = 0; i < d; i++) out[i] = oracle_bf16_value(oracle_bf16_round(x[i]));
    } else {
        (void)fp8_row(x, d, NULL, out);
    }
}

/* ------------------------------------------------------------------------ */
/* Voting (Sec. III-A).  f_t(x; q) = 1 when x lies in the leaf of tree t that */
/* q is routed to, else 0; F(x; q) = sum_t f_t(x; q); the candidate set is    */
/* S = {x : F(x; q) >= v}.  F is first summed over every tree, then S is read */
/* off the points with a nonzero F, in ascending id order.                    */
/*   F      : n counters, all zero on entry and on return                     */
/*   touched: scratch of T * max_leaf ids                                     */
/*   S, FS  : receive the members of S (ascending) and their F; returns |S|   */
/* ------------------------------------------------------------------------ */
static int64_t vote_set(const float *qv, int32_t d, int32_t T, int32_t depth, const float *R,
                        const float *splits, const int32_t *perm, int64_t n, const int64_t *off,
                        int32_t v, int32_t *F, int32_t *touched, int32_t *S, int32_t *FS,
                        int32_t *leaf_out)
{
    int64_t nsplit = ((int64_t)1 << depth) - 1;
    int64_t nt = 0;
    for (int32_t t = 0; t < T; t++) {
        int32_t L = route_one(qv, d, R + (int64_t)t * depth * d, depth, splits + (int64_t)t * nsplit);
        if (leaf_out) leaf_out[t] = L;
        const int32_t *pts = perm + (int64_t)t * n;
        for (int64_t s = off[L]; s < off[L + 1]; s++) {
            int32_t x = pts[s];
            if (F[x] == 0) touched[nt++] = x;
            F[x] += 1;                                  /* f_t(x; q) = 1 */
        }
    }
    qsort(touched, (size_t)nt, sizeof(int32_t), cmp_id);
    int64_t ns = 0;
    for (int64_t i = 0; i < nt; i++) {
        int32_t x = touched[i];
        if (F[x] >= v) {
            S[ns] = x;
            FS[ns] = F[x];
            ns++;
        }
        F[x] = 0;
    }
    return ns;
}

/* ------------------------------------------------------------------------ */
/* approximate_knn (Alg. 4) for a batch of queries.                           */
/*   off: leaf offsets (2^depth + 1), perm: T x n leaf lists.                 */
/*   s_count[q] = |S| (optional).  If s_ids is given, the candidate ids of    */
/*   query q, ascending, go to s_ids[q*s_cap ...] with their vote counts in   */
/*   s_votes (|S| must fit in s_cap).                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *X; int64_t n; int32_t d; int32_t T; int32_t depth;
    const float *R; const float *splits; const int32_t *perm; const int64_t *off;
    const float *Q; int64_t nq; int32_t k; int32_t v;
    int32_t *out_idx; double *out_dist; int64_t *s_count;
    int32_t *s_ids; int32_t *s_votes; int64_t s_cap; int32_t *leaf_out;
    /* precision arm (0: none) and its kept list */
    int32_t arm; int32_t kp; int32_t *keep_ids; double *keep_score; int32_t *keep_count;
    int64_t first, stride;
} query_job;

static int64_t max_leaf_size(const int64_t *off, int32_t depth)
{
    int64_t m = 0;
    for (int64_t L = 0; L < ((int64_t)1 << depth); L++)
        if (off[L + 1] - off[L] > m) m = off[L + 1] - off[L];
    return m;
}

/* squared Euclidean distance in float64 between q and a decoded row */
static double sq_dist_decoded(const float *q, const double *xt, int32_t d)
{
    double s = 0.0;
    for (int32_t i = 0; i < d; i++) {
        double diff = (double)q[i] - xt[i];
        s += diff * diff;
    }
    return s;
}

static void *query_worker(void *arg)
{
    query_job *j = (query_job *)arg;
    int64_t ml = max_leaf_size(j->off, j->depth);
    int64_t tcap = (int64_t)j->T * ml;
    int32_t *F = (int32_t *)calloc((size_t)j->n, sizeof(int32_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tcap > 0 ? tcap : 1));
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tcap > 0 ? tcap : 1));
    int32_t *FS = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tcap > 0 ? tcap : 1));
    cand_t *scratch = (cand_t *)malloc(sizeof(cand_t) * (size_t)(tcap > 0 ? tcap : 1));
    int32_t *kept = (int32_t *)malloc(sizeof(int32_t) * (size_t)(j->kp > 0 ? j->kp : 1));
    double *rowbuf = (double *)malloc(sizeof(double) * (size_t)j->d);
    for (int64_t q = j->first; q < j->nq; q += j->stride) {
        const float *qv = j->Q + q * j->d;
        int64_t ns = vote_set(qv, j->d, j->T, j->depth, j->R, j->splits, j->perm, j->n, j->off, j->v,
                              F, touched, S, FS, j->leaf_out ? j->leaf_out + q * j->T : NULL);
        if (j->s_count) j->s_count[q] = ns;
        if (j->s_ids) {
            int64_t m = ns < j->s_cap ? ns : j->s_cap;
            memcpy(j->s_ids + q * j->s_cap, S, sizeof(int32_t) * (size_t)m);
            if (j->s_votes) memcpy(j->s_votes + q * j->s_cap, FS, sizeof(int32_t) * (size_t)m);
        }
        if (j->arm == 0) {
            knn_in_set(qv, j->X, j->d, S, ns, j->k, scratch, j->out_idx + q * j->k, j->out_dist + q * j->k);
            continue;
        }
        /* precision arm: rank S by the squared distance to the decoded rows, */
        /* keep the first kp under (score, id), then the exact k-NN of those. */
        int64_t nk = ns < j->kp ? ns : j->kp;
        for (int64_t s = 0; s < ns; s++) {
            decode_row(j->arm, j->X + (int64_t)S[s] * j->d, j->d, rowbuf);
            scratch[s].id = S[s];
            scratch[s].dist = sq_dist_decoded(qv, rowbuf, j->d);
        }
        qsort(scratch, (size_t)ns, sizeof(cand_t), cmp_cand);
        for (int64_t r = 0; r < j->kp; r++) {
            j->keep_ids[q * j->kp + r] = r < nk ? scratch[r].id : -1;
            j->keep_score[q * j->kp + r] = r < nk ? scratch[r].dist : INFINITY;
        }
        j->keep_count[q] = (int32_t)nk;
        for (int64_t r = 0; r < nk; r++) kept[r] = scratch[r].id;
        knn_in_set(qv, j->X, j->d, kept, nk, j->k, scratch, j->out_idx + q * j->k, j->out_dist + q * j->k);
    }
    free(rowbuf); free(kept); free(scratch); free(FS); free(S); free(touched); free(F);
    return NULL;
}

static void run_query_jobs(query_job base, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > base.nq) nthreads = (int32_t)(base.nq > 0 ? base.nq : 1);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    query_job *jobs = (query_job *)malloc(sizeof(query_job) * (size_t)nthreads);
    for (int32_t w = 0; w < nthreads; w++) {
        jobs[w] = base;
        jobs[w].first = w;
        jobs[w].stride = nthreads;
        pthread_create(&th[w], NULL, query_worker, &jobs[w]);
    }
    for (int32_t w = 0; w < nthreads; w++) pthread_join(th[w], NULL);
    free(jobs); free(th);
}

void oracle_query(const float *X, int64_t n, int32_t d, int32_t T, int32_t depth,
                  const float *R, const float *splits, const int32_t *perm, const int64_t *off,
                  const float *Q, int64_t nq, int32_t k, int32_t v,
                  int32_t *out_idx, double *out_dist, int64_t *s_count,
                  int32_t *s_ids, int32_t *s_votes, int64_t s_cap, int32_t *leaf_out,
                  int32_t nthreads)
{
    query_job j;
    memset(&j, 0, sizeof(j));
    j.X = X; j.n = n; j.d = d; j.T = T; j.depth = depth; j.R = R; j.splits = splits; j.perm = perm;
    j.off = off; j.Q = Q; j.nq = nq; j.k = k; j.v = v; j.out_idx = out_idx; j.out_dist = out_dist;
    j.s_count = s_count; j.s_ids = s_ids; j.s_votes = s_votes; j.s_cap = s_cap; j.leaf_out = leaf_out;
    run_query_jobs(j, nthreads);
}

/* the precision arm of a query batch: arm 1 = bfloat16 rows, arm 2 = fp8  */
/* rows.  For each query, S is formed as in oracle_query; its members are  */
/* ranked by the squared float64 distance between q and the decoded row    */
/* (= ||q||^2 + ||x~||^2 - 2 q.x~), the first kp under (score, id) are kept */
/* (keep_ids / keep_score, kp per query, padded with -1 / +inf), and the    */
/* answer is the exact k-NN (float64, order (distance, id)) of the kept.    */
void oracle_query_prefilter(const float *X, int64_t n, int32_t d, int32_t T, int32_t depth,
                            const float *R, const float *splits, const int32_t *perm, const int64_t *off,
                            const float *Q, int64_t nq, int32_t k, int32_t v, int32_t arm, int32_t kp,
                            int32_t *out_idx, double *out_dist, int64_t *s_count,
                            int32_t *keep_ids, double *keep_score, int32_t *keep_count, int32_t nthreads)
{
    query_job j;
    memset(&j, 0, sizeof(j));
    j.X = X; j.n = n; j.d = d; j.T = T; j.depth = depth; j.R = R; j.splits = splits; j.perm = perm;
    j.off = off; j.Q = Q; j.nq = nq; j.k = k; j.v = v; j.out_idx = out_idx; j.out_dist = out_dist;
    j.s_count = s_count; j.arm = arm; j.kp = kp; j.keep_ids = keep_ids;
    j.keep_score = keep_score; j.keep_count = keep_count;
    run_query_jobs(j, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Brute-force exact k-NN (Sec. I-A): the k points of X closest to q in       */
/* float64 Euclidean distance, order (distance, id).  A sorted list of the k  */
/* best is kept by insertion.                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *X; int64_t n; int32_t d; const float *Q; int64_t nq; int32_t k;
    int32_t *out_idx; double *out_dist; int64_t first, stride;
} bf_job;

static void *bf_worker(void *arg)
{
    bf_job *j = (bf_job *)arg;
    cand_t *best = (cand_t *)malloc(sizeof(cand_t) * (size_t)(j->k + 1));
    for (int64_t q = j->first; q < j->nq; q += j->stride) {
        const float *qv = j->Q + q * j->d;
        int32_t nb = 0;
        for (int64_t x = 0; x < j->n; x++) {
            cand_t c = {oracle_distance(qv, j->X + x * j->d, j->d), (int32_t)x};
            if (nb == j->k && cmp_cand(&c, &best[nb - 1]) >= 0) continue;
            int32_t pos = nb < j->k ? nb : j->k - 1;
            if (nb < j->k) nb++;
            while (pos > 0 && cmp_cand(&c, &best[pos - 1]) < 0) {
                best[pos] = best[pos - 1];
                pos--;
            }
            best[pos] = c;
        }
        for (int32_t r = 0; r < j->k; r++) {
            if (r < nb) { j->out_idx[q * j->k + r] = best[r].id; j->out_dist[q * j->k + r] = best[r].dist; }
            else        { j->out_idx[q * j->k + r] = -1;         j->out_dist[q * j->k + r] = INFINITY; }
        }
    }
    free(best);
    return NULL;
}

void oracle_bruteforce(const float *X, int64_t n, int32_t d, const float *Q, int64_t nq, int32_t k,
                       int32_t *out_idx, double *out_dist, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nq) nthreads = (int32_t)(nq > 0 ? nq : 1);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    bf_job *jobs = (bf_job *)malloc(sizeof(bf_job) * (size_t)nthreads);
    for (int32_t w = 0; w < nthreads; w++) {
        bf_job j = {X, n, d, Q, nq, k, out_idx, out_dist, w, nthreads};
        jobs[w] = j;
        pthread_create(&th[w], NULL, bf_worker, &jobs[w]);
    }
    for (int32_t w = 0; w < nthreads; w++) pthread_join(th[w], NULL);
    free(jobs); free(th);
}
