/*
 * FP64 CPU oracle for the MLFMA near-field (P2P) operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library never
 * links, includes or calls it, and it shares no code with the GPU library.
 *
 * What it computes (arXiv 2511.21535; the paper gives no formulas for the
 * kernels, so the readings below are stated where they are used):
 *   - the near field of a leaf box is the box itself plus every leaf box whose
 *     closed cube touches it (the "order-1-box stencil", Sec. 2.2; the E2
 *     neighbourhood of Sec. 5.1);
 *   - the P2P operator is the direct pairwise sum over that near field
 *     (Sec. 1, Sec. 2.1);
 *   - the redundant layout copies, for every target box, the sources of all
 *     its near boxes into one contiguous segment (Sec. 1.1, Sec. 5.2.1);
 *   - the Locality metric is Definition 1 with Formulas (10) and (11) (Sec. 3.4).
 *
 * Everything here is the plain definition, written with plain loops, in
 * double precision, with plain (uncompensated) sums.  OpenMP only splits
 * independent targets between threads; no loop is blocked or reordered.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DEPTH_BITS 20           /* particle keys: 20 bits per axis */
#define ORC_PI 3.14159265358979323846

/* Sets the number of OpenMP threads of the parallel loops below (n >= 1). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads the parallel loops below use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Keys                                                                     */
/* ------------------------------------------------------------------------ */

/* Interleave the low `bits` bits of three integers, bit b of x going to key
 * bit 3b, of y to 3b+1, of z to 3b+2 (x is the least significant). */
uint64_t orc_morton3(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint64_t key = 0;
    for (int b = 0; b < bits; ++b) {
        key |= (uint64_t)((x >> b) & 1u) << (3 * b);
        key |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        key |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return key;
}

/* Particle keys.  c_d = floor(x_d * 2^20) for x_d in [0,1); key = Morton(c).
 * Returns the number of points outside [0,1)^3 (NaN included); their key is 0. */
int64_t orc_particle_keys(int64_t n, const double *x, const double *y, const double *z,
                          uint64_t *key)
{
    int64_t bad = 0;
    const double scale = (double)(1u << ORC_DEPTH_BITS);
    for (int64_t i = 0; i < n; ++i) {
        double p[3] = {x[i], y[i], z[i]};
        int ok = 1;
        uint32_t c[3];
        for (int d = 0; d < 3; ++d) {
            if (!(p[d] >= 0.0 && p[d] < 1.0)) { ok = 0; break; }
            c[d] = (uint32_t)floor(p[d] * scale);
        }
        if (!ok) { ++bad; key[i] = 0; continue; }
        key[i] = orc_morton3(c[0], c[1], c[2], ORC_DEPTH_BITS);
    }
    return bad;
}

/* Bits per axis of the grid key space: the smallest b >= 2 with 2^b >= every
 * edge length. */
int32_t orc_grid_bits(int32_t n_grids, const int32_t *n_side)
{
    int32_t mx = 4;
    for (int32_t g = 0; g < n_grids; ++g) if (n_side[g] > mx) mx = n_side[g];
    int32_t b = 2;
    while ((1 << b) < mx) ++b;
    return b;
}

/* Grid keys.  Instance g holds n_side[g]^3 points in caller order
 * p = point_off[g] + i + n (j + n k).  key = (g << 3b) | Morton_b(i, j, k). */
void orc_grid_keys(int32_t n_grids, const int32_t *n_side, const int64_t *point_off,
                   uint64_t *key)
{
    int32_t b = orc_grid_bits(n_grids, n_side);
    for (int32_t g = 0; g < n_grids; ++g) {
        int64_t n = n_side[g];
        for (int64_t k = 0; k < n; ++k)
            for (int64_t j = 0; j < n; ++j)
                for (int64_t i = 0; i < n; ++i) {
                    int64_t p = point_off[g] + i + n * (j + n * k);
                    key[p] = ((uint64_t)g << (3 * b)) |
                             orc_morton3((uint32_t)i, (uint32_t)j, (uint32_t)k, b);
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Tree                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t key; int64_t idx; } orc_pair;

static int orc_cmp_pair(const void *a, const void *b)
{
    const orc_pair *p = (const orc_pair *)a, *q = (const orc_pair *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

typedef struct {
    const uint64_t *skey;     /* keys in sorted order */
    int depth, leaf_cap;
    int64_t n_leaves;
    int32_t *leaf_start;
    uint64_t *leaf_key;
    int8_t *leaf_level;
    int32_t *anchor;          /* [L][3], units of 2^-20 */
    int32_t *size;            /* [L] */
} orc_build_ctx;

/* Visit the node at `level` with lower corner `a` holding sorted slots
 * [lo, hi).  Uniform trees (leaf_cap == 0) split every node above `depth`;
 * adaptive trees split a node iff it holds more than leaf_cap points and its
 * level is below `depth`.  Children are visited in child-index order
 * (bit 0 = x, bit 1 = y, bit 2 = z), empty children are dropped, so leaves
 * come out in ascending key order. */
static void orc_visit(orc_build_ctx *c, int level, const uint32_t a[3], int64_t lo, int64_t hi)
{
    if (hi <= lo) return;
    int64_t count = hi - lo;
    int split = (c->leaf_cap == 0) ? (level < c->depth)
                                   : (count > c->leaf_cap && level < c->depth);
    if (!split) {
        int64_t L = c->n_leaves++;
        c->leaf_start[L] = (int32_t)lo;
        c->leaf_level[L] = (int8_t)level;
        c->leaf_key[L] = orc_morton3(a[0], a[1], a[2], ORC_DEPTH_BITS);
        c->anchor[3 * L + 0] = (int32_t)a[0];
        c->anchor[3 * L + 1] = (int32_t)a[1];
        c->anchor[3 * L + 2] = (int32_t)a[2];
        c->size[L] = 1 << (ORC_DEPTH_BITS - level);
        return;
    }
    int shift = 3 * (ORC_DEPTH_BITS - level - 1);
    uint32_t half = 1u << (ORC_DEPTH_BITS - level - 1);
    int64_t pos = lo;
    for (int ch = 0; ch < 8; ++ch) {
        int64_t end = pos;
        while (end < hi && (int)((c->skey[end] >> shift) & 7u) == ch) ++end;
        uint32_t b[3] = {a[0] + (uint32_t)(ch & 1) * half,
                         a[1] + (uint32_t)((ch >> 1) & 1) * half,
                         a[2] + (uint32_t)((ch >> 2) & 1) * half};
        orc_visit(c, level + 1, b, pos, end);
        pos = end;
    }
}

/* Particle octree.  perm = caller indices sorted stably by (key, index).
 * Returns the number of leaves L; leaf_start has L+1 entries.  Arrays must
 * hold n entries (L <= n). */
int64_t orc_build_tree_particles(int64_t n, const uint64_t *key, int32_t depth, int32_t leaf_cap,
                                 int32_t *perm, int32_t *leaf_start, uint64_t *leaf_key,
                                 int8_t *leaf_level, int32_t *anchor, int32_t *size)
{
    orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
    uint64_t *sk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { pr[i].key = key[i]; pr[i].idx = i; }
    qsort(pr, (size_t)n, sizeof(orc_pair), orc_cmp_pair);
    for (int64_t i = 0; i < n; ++i) { perm[i] = (int32_t)pr[i].idx; sk[i] = pr[i].key; }
    orc_build_ctx c = {sk, depth, leaf_cap, 0, leaf_start, leaf_key, leaf_level, anchor, size};
    uint32_t root[3] = {0, 0, 0};
    orc_visit(&c, 0, root, 0, n);
    leaf_start[c.n_leaves] = (int32_t)n;
    free(pr);
    free(sk);
    return c.n_leaves;
}

/* Grid "tree": the leaves are the boxes of 4x4x4 points of every instance.
 * perm = caller indices sorted by key; a leaf is a maximal run of equal
 * key >> 6.  anchor = (i, j, k) of the box's lowest point (point units),
 * size = 4, inst = instance, level = b - 2.  Returns L. */
int64_t orc_build_tree_grids(int32_t n_grids, const int32_t *n_side, const int64_t *point_off,
                             int64_t n, const uint64_t *key,
                             int32_t *perm, int32_t *leaf_start, uint64_t *leaf_key,
                             int8_t *leaf_level, int32_t *anchor, int32_t *size, int32_t *inst)
{
    int32_t b = orc_grid_bits(n_grids, n_side);
    orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { pr[i].key = key[i]; pr[i].idx = i; }
    qsort(pr, (size_t)n, sizeof(orc_pair), orc_cmp_pair);
    int64_t L = 0;
    for (int64_t s = 0; s < n; ++s) {
        perm[s] = (int32_t)pr[s].idx;
        if (s == 0 || (pr[s].key >> 6) != (pr[s - 1].key >> 6)) {
            int64_t p = pr[s].idx;
            int32_t g = 0;
            while (g + 1 < n_grids && point_off[g + 1] <= p) ++g;
            int64_t ns = n_side[g], loc = p - point_off[g];
            int64_t i = loc % ns, j = (loc / ns) % ns, k = loc / (ns * ns);
            leaf_start[L] = (int32_t)s;
            leaf_key[L] = pr[s].key;
            leaf_level[L] = (int8_t)(b - 2);
            anchor[3 * L + 0] = (int32_t)i;
            anchor[3 * L + 1] = (int32_t)j;
            anchor[3 * L + 2] = (int32_t)k;
            size[L] = 4;
            inst[L] = g;
            ++L;
        }
    }
    leaf_start[L] = (int32_t)n;
    free(pr);
    return L;
}

/* ------------------------------------------------------------------------ */
/* Near-field lists                                                         */
/* ------------------------------------------------------------------------ */

/* Closed cubes [a, a+sa] and [b, b+sb] touch or overlap on every axis. */
static int orc_adjacent(const int32_t *a, int32_t sa, const int32_t *b, int32_t sb)
{
    for (int d = 0; d < 3; ++d) {
        int64_t ad = a[d], bd = b[d];
        if (!(ad <= bd + sb && bd <= ad + sa)) return 0;
    }
    return 1;
}

/* Near lists of the leaves listed in `targets` (brute force over all L
 * leaves).  nbr(A) = every leaf B (of the same instance, if inst != NULL)
 * whose closed cube touches A's, A included, in ascending leaf id.
 * Writes nbr_start[0..n_targets] and, if the total fits in `cap`, nbr_idx.
 * Returns the total number of entries. */
int64_t orc_neighbors(int64_t L, const int32_t *anchor, const int32_t *size, const int32_t *inst,
                      const int32_t *targets, int64_t n_targets,
                      int64_t *nbr_start, int32_t *nbr_idx, int64_t cap)
{
    int64_t *cnt = (int64_t *)calloc((size_t)(n_targets + 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_targets; ++t) {
        int32_t A = targets[t];
        int64_t c = 0;
        for (int64_t B = 0; B < L; ++B) {
            if (inst && inst[B] != inst[A]) continue;
            if (orc_adjacent(&anchor[3 * A], size[A], &anchor[3 * B], size[B])) ++c;
        }
        cnt[t] = c;
    }
    nbr_start[0] = 0;
    for (int64_t t = 0; t < n_targets; ++t) nbr_start[t + 1] = nbr_start[t] + cnt[t];
    int64_t total = nbr_start[n_targets];
    if (total <= cap && nbr_idx) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < n_targets; ++t) {
            int32_t A = targets[t];
            int64_t w = nbr_start[t];
            for (int64_t B = 0; B < L; ++B) {
                if (inst && inst[B] != inst[A]) continue;
                if (orc_adjacent(&anchor[3 * A], size[A], &anchor[3 * B], size[B]))
                    nbr_idx[w++] = (int32_t)B;
            }
        }
    }
    free(cnt);
    return total;
}

/* Periodic images (the periodic interactions of the stellar-dynamics case,
 * Sec. 5.2): image code c = (sx+1) + 3 (sy+1) + 9 (sz+1), sx, sy, sz in
 * {-1, 0, 1}, shifts a source by (sx, sy, sz) domain edges; code 13 is no
 * shift.  A NULL shift array means code 13 for every entry. */
static void orc_shift_of(const int8_t *shift, int64_t e, double s[3])
{
    int c = shift ? shift[e] : 13;
    s[0] = (double)(c % 3 - 1);
    s[1] = (double)((c / 3) % 3 - 1);
    s[2] = (double)(c / 9 - 1);
}

static int orc_shift_code(const int8_t *shift, int64_t e) { return shift ? shift[e] : 13; }

/* Periodic near lists of the leaves listed in `targets` (particles, unit
 * torus): nbr(A) = every (leaf B, image c) whose closed cube, shifted by
 * image c, touches A's, in ascending (c, B).  Writes nbr_start and, if the
 * total fits in `cap`, nbr_idx and nbr_shift.  Returns the entry count. */
int64_t orc_neighbors_periodic(int64_t L, const int32_t *anchor, const int32_t *size,
                               const int32_t *targets, int64_t n_targets, int64_t *nbr_start,
                               int32_t *nbr_idx, int8_t *nbr_shift, int64_t cap)
{
    const int64_t dim = (int64_t)1 << ORC_DEPTH_BITS;
    int64_t *cnt = (int64_t *)calloc((size_t)(n_targets + 1), sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            nbr_start[0] = 0;
            for (int64_t t = 0; t < n_targets; ++t) nbr_start[t + 1] = nbr_start[t] + cnt[t];
            if (nbr_start[n_targets] > cap || !nbr_idx) break;
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < n_targets; ++t) {
            int32_t A = targets[t];
            int64_t c = 0, w = pass ? nbr_start[t] : 0;
            for (int code = 0; code < 27; ++code) {
                int64_t sh[3] = {(code % 3 - 1) * dim, ((code / 3) % 3 - 1) * dim, (code / 9 - 1) * dim};
                for (int64_t B = 0; B < L; ++B) {
                    int adj = 1;
                    for (int d = 0; d < 3; ++d) {
                        int64_t ad = anchor[3 * A + d], bd = anchor[3 * B + d] + sh[d];
                        if (!(ad <= bd + size[B] && bd <= ad + size[A])) adj = 0;
                    }
                    if (!adj) continue;
                    if (pass) {
                        nbr_idx[w] = (int32_t)B;
                        nbr_shift[w] = (int8_t)code;
                        ++w;
                    } else {
                        ++c;
                    }
                }
            }
            if (!pass) cnt[t] = c;
        }
    }
    int64_t total = nbr_start[n_targets];
    free(cnt);
    return total;
}

/* Remote near lists (the remote interactions of the stellar-dynamics case,
 * Sec. 5.2: sources received from another domain): for every leaf A of the
 * target tree (Lt leaves), every leaf B of a second, source tree (Ls leaves,
 * another particle set in the same unit cube) whose closed cube touches A's;
 * with periodic != 0 also through the 26 shifted images (codes as in
 * orc_neighbors_periodic), else code 13 only.  Entries in ascending (code, B).
 * Writes nbr_start and, if the total fits in `cap`, nbr_idx and nbr_shift
 * (which may be NULL).  Returns the entry count. */
int64_t orc_neighbors_cross(int64_t Lt, const int32_t *t_anchor, const int32_t *t_size, int64_t Ls,
                            const int32_t *s_anchor, const int32_t *s_size, int32_t periodic,
                            int64_t *nbr_start, int32_t *nbr_idx, int8_t *nbr_shift, int64_t cap)
{
    const int64_t dim = (int64_t)1 << ORC_DEPTH_BITS;
    int64_t *cnt = (int64_t *)calloc((size_t)(Lt + 1), sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            nbr_start[0] = 0;
            for (int64_t A = 0; A < Lt; ++A) nbr_start[A + 1] = nbr_start[A] + cnt[A];
            if (nbr_start[Lt] > cap || !nbr_idx) break;
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t A = 0; A < Lt; ++A) {
            int64_t c = 0, w = pass ? nbr_start[A] : 0;
            for (int code = periodic ? 0 : 13; code <= (periodic ? 26 : 13); ++code) {
                int64_t sh[3] = {(code % 3 - 1) * dim, ((code / 3) % 3 - 1) * dim, (code / 9 - 1) * dim};
                for (int64_t B = 0; B < Ls; ++B) {
                    int adj = 1;
                    for (int d = 0; d < 3; ++d) {
                        int64_t ad = t_anchor[3 * A + d], bd = s_anchor[3 * B + d] + sh[d];
                        if (!(ad <= bd + s_size[B] && bd <= ad + t_size[A])) adj = 0;
                    }
                    if (!adj) continue;
                    if (pass) {
                        nbr_idx[w] = (int32_t)B;
                        if (nbr_shift) nbr_shift[w] = (int8_t)code;
                        ++w;
                    } else {
                        ++c;
                    }
                }
            }
            if (!pass) cnt[A] = c;
        }
    }
    int64_t total = nbr_start[Lt];
    free(cnt);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Redundant layout                                                         */
/* ------------------------------------------------------------------------ */

/* Segment bookkeeping for the redundant layout over all L leaves:
 * red_start = exclusive prefix sum of the segment lengths
 * sum_{B in nbr(A)} occ(B); red_self[A] = offset of A's own sources (the
 * unshifted image) inside its segment.  Returns S = red_start[L]. */
int64_t orc_red_offsets(int64_t L, const int32_t *leaf_start, const int64_t *nbr_start,
                        const int32_t *nbr_idx, const int8_t *nbr_shift, int64_t *red_start,
                        int32_t *red_self)
{
    red_start[0] = 0;
    for (int64_t A = 0; A < L; ++A) {
        int64_t len = 0, self = -1;
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            int32_t B = nbr_idx[e];
            if (B == A && orc_shift_code(nbr_shift, e) == 13) self = len;
            len += leaf_start[B + 1] - leaf_start[B];
        }
        red_start[A + 1] = red_start[A] + len;
        red_self[A] = (int32_t)self;
    }
    return red_start[L];
}

/* Redundant payload: for A in ascending order, for B in nbr(A) in order, the
 * rows src[perm[s]] of B's sorted slots s, each `row_bytes` bytes, copied
 * bit for bit. */
void orc_restructure_rows(int64_t L, const int32_t *leaf_start, const int32_t *perm,
                          const int64_t *nbr_start, const int32_t *nbr_idx,
                          const int64_t *red_start, const void *src, int64_t row_bytes, void *out)
{
    const char *s8 = (const char *)src;
    char *o8 = (char *)out;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t A = 0; A < L; ++A) {
        int64_t w = red_start[A];
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            int32_t B = nbr_idx[e];
            for (int32_t s = leaf_start[B]; s < leaf_start[B + 1]; ++s) {
                memcpy(o8 + w * row_bytes, s8 + (int64_t)perm[s] * row_bytes, (size_t)row_bytes);
                ++w;
            }
        }
    }
}

/* FP64 gravity payload: the rows (x + s, y + s, z + s, m) of the segments,
 * s the image shift of the entry (zero without images).  out8: double[S][4]. */
void orc_restructure_gravity_rows(int64_t L, const int32_t *leaf_start, const int32_t *perm,
                                  const int64_t *nbr_start, const int32_t *nbr_idx,
                                  const int8_t *nbr_shift, const int64_t *red_start,
                                  const double *x, const double *y, const double *z,
                                  const double *m, double *out8)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t A = 0; A < L; ++A) {
        int64_t w = red_start[A];
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            int32_t B = nbr_idx[e];
            double sh[3];
            orc_shift_of(nbr_shift, e, sh);
            for (int32_t s = leaf_start[B]; s < leaf_start[B + 1]; ++s, ++w) {
                int64_t j = perm[s];
                out8[4 * w + 0] = x[j] + sh[0];
                out8[4 * w + 1] = y[j] + sh[1];
                out8[4 * w + 2] = z[j] + sh[2];
                out8[4 * w + 3] = m[j];
            }
        }
    }
}

/* FP32-mixed gravity payload of the redundant layout: for target leaf A with
 * centre c_A = (anchor_A + size_A / 2) 2^-20 (exact in double), every source
 * row of its segment becomes (float)(x - c_A), (float)(y - c_A),
 * (float)(z - c_A), (float)m: the offset removed in double, the result
 * rounded to single; a source of image c is shifted first, in double
 * ((x + s) - c_A).  out4: float[S][4]. */
void orc_restructure_gravity_rel(int64_t L, const int32_t *leaf_start, const int32_t *perm,
                                 const int64_t *nbr_start, const int32_t *nbr_idx,
                                 const int8_t *nbr_shift, const int64_t *red_start,
                                 const int32_t *anchor, const int32_t *size, const double *x,
                                 const double *y, const double *z, const double *m, float *out4)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t A = 0; A < L; ++A) {
        double c[3];
        for (int d = 0; d < 3; ++d)
            c[d] = ((double)anchor[3 * A + d] + 0.5 * (double)size[A]) / (double)(1u << ORC_DEPTH_BITS);
        int64_t w = red_start[A];
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            int32_t B = nbr_idx[e];
            double sh[3];
            orc_shift_of(nbr_shift, e, sh);
            for (int32_t s = leaf_start[B]; s < leaf_start[B + 1]; ++s) {
                int64_t j = perm[s];
                out4[4 * w + 0] = (float)((x[j] + sh[0]) - c[0]);
                out4[4 * w + 1] = (float)((y[j] + sh[1]) - c[1]);
                out4[4 * w + 2] = (float)((z[j] + sh[2]) - c[2]);
                out4[4 * w + 3] = (float)m[j];
                ++w;
            }
        }
    }
}

/* Per-interaction (thread-level) layout of the stellar-dynamics case (Sec.
 * 5.2.1): one record per near-list entry e = (A, B) in list order -- a header
 * row (occ_A, occ_B, A, B), then the rows of A's sorted slots (the targets),
 * then the rows of B's sorted slots (the sources).  rec_start[0..E] receives
 * the record offsets; the total row count is returned.  With out8 != NULL the
 * rows are double[4] (x, y, z, m) and the header holds the integers as
 * doubles; with out4 != NULL they are float[4] relative to the centre of A,
 * as in orc_restructure_gravity_rel, and the header holds the int32 bit
 * patterns.  Either output may be NULL (offsets only). */
int64_t orc_restructure_interactions(int64_t L, const int32_t *leaf_start, const int32_t *perm,
                                     const int64_t *nbr_start, const int32_t *nbr_idx,
                                     const int8_t *nbr_shift, const int32_t *anchor, const int32_t *size,
                                     const double *x, const double *y, const double *z,
                                     const double *m, int64_t *rec_start, double *out8,
                                     float *out4)
{
    int64_t E = nbr_start[L], w = 0;
    for (int64_t A = 0; A < L; ++A) {
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            int32_t B = nbr_idx[e];
            rec_start[e] = w;
            w += 1 + (leaf_start[A + 1] - leaf_start[A]) + (leaf_start[B + 1] - leaf_start[B]);
        }
    }
    rec_start[E] = w;
    if (!out8 && !out4) return w;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t A = 0; A < L; ++A) {
        double c[3];
        for (int d = 0; d < 3; ++d)
            c[d] = ((double)anchor[3 * A + d] + 0.5 * (double)size[A]) / (double)(1u << ORC_DEPTH_BITS);
        int32_t occA = leaf_start[A + 1] - leaf_start[A];
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            int32_t B = nbr_idx[e];
            int32_t occB = leaf_start[B + 1] - leaf_start[B];
            int64_t r = rec_start[e];
            int32_t hdr[4] = {occA, occB, (int32_t)A, B};
            if (out8)
                for (int k = 0; k < 4; ++k) out8[4 * r + k] = (double)hdr[k];
            if (out4)
                memcpy(&out4[4 * r], hdr, sizeof(hdr));
            ++r;
            /* the targets (A's slots), then the sources (B's slots, shifted by
             * the entry's image) */
            for (int part = 0; part < 2; ++part) {
                int32_t lo = part == 0 ? leaf_start[A] : leaf_start[B];
                int32_t hi = part == 0 ? leaf_start[A + 1] : leaf_start[B + 1];
                double sh[3] = {0.0, 0.0, 0.0};
                if (part == 1) orc_shift_of(nbr_shift, e, sh);
                for (int32_t sl = lo; sl < hi; ++sl, ++r) {
                    int64_t j = perm[sl];
                    if (out8) {
                        out8[4 * r + 0] = x[j] + sh[0];
                        out8[4 * r + 1] = y[j] + sh[1];
                        out8[4 * r + 2] = z[j] + sh[2];
                        out8[4 * r + 3] = m[j];
                    }
                    if (out4) {
                        out4[4 * r + 0] = (float)((x[j] + sh[0]) - c[0]);
                        out4[4 * r + 1] = (float)((y[j] + sh[1]) - c[1]);
                        out4[4 * r + 2] = (float)((z[j] + sh[2]) - c[2]);
                        out4[4 * r + 3] = (float)m[j];
                    }
                }
            }
        }
    }
    return w;
}

/* ------------------------------------------------------------------------ */
/* Gravity                                                                  */
/* ------------------------------------------------------------------------ */

/* Plummer-softened Newtonian gravity with G = 1 over the near field:
 *   phi_i = - sum_{j near i, j != i} m_j (r_ij^2 + eps^2)^{-1/2}
 *   a_i   = - sum_{j near i, j != i} m_j (x_i - x_j) (r_ij^2 + eps^2)^{-3/2}
 * For the selected leaves sel[0..n_sel) with near lists (sel_nbr_start,
 * sel_nbr_idx) -- list k belongs to sel[k] -- the targets are the particles
 * of those leaves, in sorted-slot order.  out_idx receives their caller
 * indices; phi/ax/ay/az the values.  Returns the number of targets.
 * With eps == 0 a coincident pair i != j gives inf/nan, as the formula does.
 * sel_nbr_shift (may be NULL) gives each entry's periodic image: the source
 * then sits at x_j + s, and only the unshifted image of i itself is skipped. */
int64_t orc_gravity_leaves(const double *x, const double *y, const double *z, const double *m,
                           double eps, const int32_t *perm, const int32_t *leaf_start,
                           const int32_t *sel, int64_t n_sel,
                           const int64_t *sel_nbr_start, const int32_t *sel_nbr_idx,
                           const int8_t *sel_nbr_shift,
                           int32_t *out_idx, double *phi, double *ax, double *ay, double *az)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_sel + 1));
    off[0] = 0;
    for (int64_t k = 0; k < n_sel; ++k)
        off[k + 1] = off[k] + (leaf_start[sel[k] + 1] - leaf_start[sel[k]]);
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < n_sel; ++k) {
        int32_t A = sel[k];
        for (int32_t s = leaf_start[A]; s < leaf_start[A + 1]; ++s) {
            int64_t i = perm[s];
            double p = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
            for (int64_t e = sel_nbr_start[k]; e < sel_nbr_start[k + 1]; ++e) {
                int32_t B = sel_nbr_idx[e];
                double sh[3];
                orc_shift_of(sel_nbr_shift, e, sh);
                int self_image = orc_shift_code(sel_nbr_shift, e) == 13;
                for (int32_t t = leaf_start[B]; t < leaf_start[B + 1]; ++t) {
                    int64_t j = perm[t];
                    if (j == i && self_image) continue;
                    double dx = x[i] - (x[j] + sh[0]), dy = y[i] - (y[j] + sh[1]), dz = z[i] - (z[j] + sh[2]);
                    double r2 = dx * dx + dy * dy + dz * dz + eps2;
                    double w = 1.0 / sqrt(r2);
                    double w3 = w * w * w;
                    p -= m[j] * w;
                    gx -= m[j] * w3 * dx;
                    gy -= m[j] * w3 * dy;
                    gz -= m[j] * w3 * dz;
                }
            }
            int64_t o = off[k] + (s - leaf_start[A]);
            out_idx[o] = (int32_t)i;
            phi[o] = p; ax[o] = gx; ay[o] = gy; az[o] = gz;
        }
    }
    int64_t total = off[n_sel];
    free(off);
    return total;
}

/* Remote gravity: for every target point i (caller order of the target set,
 * n_t points, tree (t_perm, t_leaf_start) with Lt leaves), the sums of
 * orc_gravity_leaves over the source points j of the leaves in its leaf's
 * remote list (source set sx, sy, sz, sm, tree (s_perm, s_leaf_start)), each
 * at its image x_j + s.  The two sets are distinct, so no pair is skipped.
 * Writes phi, ax, ay, az [n_t]. */
void orc_gravity_remote(int64_t Lt, const int32_t *t_perm, const int32_t *t_leaf_start,
                        const double *tx, const double *ty, const double *tz,
                        const int32_t *s_perm, const int32_t *s_leaf_start, const double *sx,
                        const double *sy, const double *sz, const double *sm, double eps,
                        const int64_t *nbr_start, const int32_t *nbr_idx, const int8_t *nbr_shift,
                        double *phi, double *ax, double *ay, double *az)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t A = 0; A < Lt; ++A) {
        for (int32_t s = t_leaf_start[A]; s < t_leaf_start[A + 1]; ++s) {
            int64_t i = t_perm[s];
            double p = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
            for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
                int32_t B = nbr_idx[e];
                double sh[3];
                orc_shift_of(nbr_shift, e, sh);
                for (int32_t t = s_leaf_start[B]; t < s_leaf_start[B + 1]; ++t) {
                    int64_t j = s_perm[t];
                    double dx = tx[i] - (sx[j] + sh[0]), dy = ty[i] - (sy[j] + sh[1]), dz = tz[i] - (sz[j] + sh[2]);
                    double r2 = dx * dx + dy * dy + dz * dz + eps2;
                    double w = 1.0 / sqrt(r2);
                    double w3 = w * w * w;
                    p -= sm[j] * w;
                    gx -= sm[j] * w3 * dx;
                    gy -= sm[j] * w3 * dy;
                    gz -= sm[j] * w3 * dz;
                }
            }
            phi[i] = p; ax[i] = gx; ay[i] = gy; az[i] = gz;
        }
    }
}

/* Reverse-mode derivative of the gravity sums.  With upstream gradients
 * (gp_i, ga_i) of phi_i and a_i, one pair (target i, source j) contributes
 *   T_ij = - m_j [ gp_i w + w^3 (ga_i . d) ],   d = x_i - x_j,
 *   w = (|d|^2 + eps^2)^{-1/2},
 * to L = sum_i gp_i phi_i + ga_i . a_i.  Its partial derivatives are
 *   dT/dm_j = - [ gp_i w + w^3 (ga_i . d) ]
 *   dT/dd   =   m_j [ gp_i w^3 d + 3 w^5 (ga_i . d) d - w^3 ga_i ]
 * with dT/dx_i = dT/dd and dT/dx_j = -dT/dd.  The near relation is symmetric,
 * so the pairs that involve particle j are (j, k) and (k, j) for k in the
 * near field of j.  For the particles of the selected leaves this sums
 *   gm_j = sum_k dT_kj/dm_j,   gx_j = sum_k [ dT_jk/dx_j + dT_kj/dx_j ].
 * Outputs follow the sorted-slot order of the selected leaves, as in
 * orc_gravity_leaves.  Returns the number of outputs. */
int64_t orc_gravity_adjoint_leaves(const double *x, const double *y, const double *z,
                                   const double *m, double eps,
                                   const double *gp, const double *gax, const double *gay,
                                   const double *gaz,
                                   const int32_t *perm, const int32_t *leaf_start,
                                   const int32_t *sel, int64_t n_sel,
                                   const int64_t *sel_nbr_start, const int32_t *sel_nbr_idx,
                                   const int8_t *sel_nbr_shift,
                                   int32_t *out_idx, double *gm, double *gx, double *gy,
                                   double *gz)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_sel + 1));
    off[0] = 0;
    for (int64_t k = 0; k < n_sel; ++k)
        off[k + 1] = off[k] + (leaf_start[sel[k] + 1] - leaf_start[sel[k]]);
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < n_sel; ++k) {
        int32_t A = sel[k];
        for (int32_t s = leaf_start[A]; s < leaf_start[A + 1]; ++s) {
            int64_t j = perm[s];
            double om = 0.0, ox = 0.0, oy = 0.0, oz = 0.0;
            for (int64_t e = sel_nbr_start[k]; e < sel_nbr_start[k + 1]; ++e) {
                int32_t B = sel_nbr_idx[e];
                double sh[3];
                orc_shift_of(sel_nbr_shift, e, sh);
                int self_image = orc_shift_code(sel_nbr_shift, e) == 13;
                for (int32_t t = leaf_start[B]; t < leaf_start[B + 1]; ++t) {
                    int64_t q = perm[t];
                    if (q == j && self_image) continue;
                    /* q's image at x_q + s; the reverse pair (target q, source j)
                     * sees j's image at x_j - s, so both use d = x_j - (x_q + s) */
                    /* pair (target j, source q): derivative w.r.t. x_j = dT/dd */
                    {
                        double d[3] = {x[j] - (x[q] + sh[0]), y[j] - (y[q] + sh[1]), z[j] - (z[q] + sh[2])};
                        double g[3] = {gax[j], gay[j], gaz[j]};
                        double w = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2);
                        double w3 = w * w * w, w5 = w3 * w * w;
                        double gd = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
                        double dd[3];
                        for (int c = 0; c < 3; ++c)
                            dd[c] = m[q] * (gp[j] * w3 * d[c] + 3.0 * w5 * gd * d[c] - w3 * g[c]);
                        ox += dd[0]; oy += dd[1]; oz += dd[2];
                    }
                    /* pair (target q, source j): derivatives w.r.t. m_j and x_j = -dT/dd */
                    {
                        double d[3] = {(x[q] + sh[0]) - x[j], (y[q] + sh[1]) - y[j], (z[q] + sh[2]) - z[j]};
                        double g[3] = {gax[q], gay[q], gaz[q]};
                        double w = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2);
                        double w3 = w * w * w, w5 = w3 * w * w;
                        double gd = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
                        om += -(gp[q] * w + w3 * gd);
                        double dd[3];
                        for (int c = 0; c < 3; ++c)
                            dd[c] = m[j] * (gp[q] * w3 * d[c] + 3.0 * w5 * gd * d[c] - w3 * g[c]);
                        ox -= dd[0]; oy -= dd[1]; oz -= dd[2];
                    }
                }
            }
            int64_t o = off[k] + (s - leaf_start[A]);
            out_idx[o] = (int32_t)j;
            gm[o] = om; gx[o] = ox; gy[o] = oy; gz[o] = oz;
        }
    }
    int64_t total = off[n_sel];
    free(off);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Helmholtz on regular grids                                               */
/* ------------------------------------------------------------------------ */

/* Locate caller index p: instance g and integer coordinates (i, j, k). */
static void orc_grid_locate(int32_t n_grids, const int32_t *n_side, const int64_t *point_off,
                            int64_t p, int32_t *g, int64_t c[3])
{
    int32_t gg = 0;
    while (gg + 1 < n_grids && point_off[gg + 1] <= p) ++gg;
    int64_t ns = n_side[gg], loc = p - point_off[gg];
    c[0] = loc % ns; c[1] = (loc / ns) % ns; c[2] = loc / (ns * ns);
    *g = gg;
}

/* Free-space Helmholtz Green's function e^{ikr}/(4 pi r) with r = h sqrt(dd)
 * for an integer squared index distance dd > 0 (e^{-i omega t} convention). */
static void orc_green(double h, double kw, int64_t dd, double *gr, double *gi)
{
    double r = h * sqrt((double)dd);
    double a = 1.0 / (4.0 * ORC_PI * r);
    *gr = cos(kw * r) * a;
    *gi = sin(kw * r) * a;
}

/* u_I = sum_{J near I, J != I} G(r_IJ) q_J for every right-hand side, where
 * J is near I when the 4x4x4 boxes holding I and J are equal or adjacent
 * (within the same instance).  Points sit at ((i+0.5)h, (j+0.5)h, (k+0.5)h).
 * q and u are complex128 stored as interleaved (re, im) pairs, q as [N][nrhs]
 * in caller order, u as [n_targets][nrhs] for the listed targets. */
void orc_helmholtz(int32_t n_grids, const int32_t *n_side, const double *h, const double *kw,
                   const int64_t *point_off, int32_t nrhs, const double *q,
                   const int64_t *targets, int64_t n_targets, double *u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t p = targets[t];
        int32_t g;
        int64_t c[3];
        orc_grid_locate(n_grids, n_side, point_off, p, &g, c);
        int64_t ns = n_side[g], nb = ns / 4;
        int64_t bx = c[0] / 4, by = c[1] / 4, bz = c[2] / 4;
        double *ur = u + 2 * t * nrhs;
        for (int32_t r = 0; r < 2 * nrhs; ++r) ur[r] = 0.0;
        for (int64_t sz = bz - 1; sz <= bz + 1; ++sz)
            for (int64_t sy = by - 1; sy <= by + 1; ++sy)
                for (int64_t sx = bx - 1; sx <= bx + 1; ++sx) {
                    if (sx < 0 || sy < 0 || sz < 0 || sx >= nb || sy >= nb || sz >= nb) continue;
                    for (int64_t k = 4 * sz; k < 4 * sz + 4; ++k)
                        for (int64_t j = 4 * sy; j < 4 * sy + 4; ++j)
                            for (int64_t i = 4 * sx; i < 4 * sx + 4; ++i) {
                                int64_t src = point_off[g] + i + ns * (j + ns * k);
                                if (src == p) continue;
                                int64_t dd = (c[0] - i) * (c[0] - i) + (c[1] - j) * (c[1] - j) +
                                             (c[2] - k) * (c[2] - k);
                                double gr, gi;
                                orc_green(h[g], kw[g], dd, &gr, &gi);
                                const double *qs = q + 2 * src * nrhs;
                                for (int32_t r = 0; r < nrhs; ++r) {
                                    ur[2 * r] += gr * qs[2 * r] - gi * qs[2 * r + 1];
                                    ur[2 * r + 1] += gr * qs[2 * r + 1] + gi * qs[2 * r];
                                }
                            }
                }
    }
}

/* Transpose action (A^T g)_J = sum_I A_IJ g_I over every target I and every
 * source J in its near field, J != I, accumulated by scattering into J.
 * Serial; for small grids.  g, out: complex128 [N][nrhs] interleaved. */
void orc_helmholtz_transpose(int32_t n_grids, const int32_t *n_side, const double *h,
                             const double *kw, const int64_t *point_off, int64_t n,
                             int32_t nrhs, const double *g, double *out)
{
    memset(out, 0, sizeof(double) * 2 * (size_t)n * (size_t)nrhs);
    for (int64_t p = 0; p < n; ++p) {
        int32_t gi_;
        int64_t c[3];
        orc_grid_locate(n_grids, n_side, point_off, p, &gi_, c);
        int64_t ns = n_side[gi_], nb = ns / 4;
        int64_t bx = c[0] / 4, by = c[1] / 4, bz = c[2] / 4;
        const double *gp = g + 2 * p * nrhs;
        for (int64_t sz = bz - 1; sz <= bz + 1; ++sz)
            for (int64_t sy = by - 1; sy <= by + 1; ++sy)
                for (int64_t sx = bx - 1; sx <= bx + 1; ++sx) {
                    if (sx < 0 || sy < 0 || sz < 0 || sx >= nb || sy >= nb || sz >= nb) continue;
                    for (int64_t k = 4 * sz; k < 4 * sz + 4; ++k)
                        for (int64_t j = 4 * sy; j < 4 * sy + 4; ++j)
                            for (int64_t i = 4 * sx; i < 4 * sx + 4; ++i) {
                                int64_t src = point_off[gi_] + i + ns * (j + ns * k);
                                if (src == p) continue;
                                int64_t dd = (c[0] - i) * (c[0] - i) + (c[1] - j) * (c[1] - j) +
                                             (c[2] - k) * (c[2] - k);
                                double gr, gim;
                                orc_green(h[gi_], kw[gi_], dd, &gr, &gim);
                                double *o = out + 2 * src * nrhs;
                                for (int32_t r = 0; r < nrhs; ++r) {
                                    o[2 * r] += gr * gp[2 * r] - gim * gp[2 * r + 1];
                                    o[2 * r + 1] += gr * gp[2 * r + 1] + gim * gp[2 * r];
                                }
                            }
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Block-level redundancy on grid trees (Sec. 3.5)                          */
/* ------------------------------------------------------------------------ */

static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* For dense, regular distributions Sec. 3.5 duplicates data per thread block
 * instead of per thread.  Here the block is a tile of grid boxes: box (i, j, k)
 * of an instance (the indices of its first point divided by 4) belongs to tile
 * (i / grain, j / grain, k / grain) of that instance.  Tiles are numbered in
 * ascending order of their smallest box id, tile_first[t] being that id.  The
 * halo of tile t is the union of the near lists of its boxes, in ascending box
 * id: halo_idx[halo_start[t] .. halo_start[t+1]).  The tile's segment holds
 * the rows of its halo boxes in that order, from row seg_start[t] on (rows =
 * sorted slots, so a box contributes its occupancy).  For entry e = (A, B) of
 * A's near list, red_row[e] is the first row of B in the segment of A's tile.
 * grain = 1 gives the box-grain segments.  Writes tile_first, halo_start and
 * seg_start (n_tiles + 1 entries each, capacity L + 1) and, if the halo total
 * fits in `cap`, halo_idx and red_row.  Returns n_tiles; *halo_total = H. */
int64_t orc_tile_layout(int64_t L, const int32_t *anchor, const int32_t *inst, const int32_t *leaf_start,
                        int32_t grain, const int64_t *nbr_start, const int32_t *nbr_idx,
                        int32_t *tile_first, int64_t *halo_start, int64_t *seg_start,
                        int32_t *halo_idx, int64_t *red_row, int64_t cap, int64_t *halo_total)
{
    /* group the boxes by tile key; a group's first box is its smallest id */
    orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(L > 0 ? L : 1));
    for (int64_t A = 0; A < L; ++A) {
        uint64_t g = inst ? (uint64_t)inst[A] : 0;
        uint64_t ti = (uint64_t)(anchor[3 * A + 0] / 4 / grain);
        uint64_t tj = (uint64_t)(anchor[3 * A + 1] / 4 / grain);
        uint64_t tk = (uint64_t)(anchor[3 * A + 2] / 4 / grain);
        pr[A].key = ((g * 1024u + ti) * 1024u + tj) * 1024u + tk;
        pr[A].idx = A;
    }
    qsort(pr, (size_t)L, sizeof(orc_pair), orc_cmp_pair);
    int64_t *tile_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L > 0 ? L : 1));
    orc_pair *first = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(L > 0 ? L : 1));
    int64_t T = 0;
    for (int64_t s = 0; s < L; ++s) {
        if (s == 0 || pr[s].key != pr[s - 1].key) {
            first[T].key = (uint64_t)pr[s].idx;   /* sorted by (key, idx): the smallest id */
            first[T].idx = T;
            ++T;
        }
    }
    /* tiles in ascending order of their first box */
    qsort(first, (size_t)T, sizeof(orc_pair), orc_cmp_pair);
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
    for (int64_t t = 0; t < T; ++t) { rank[first[t].idx] = t; tile_first[t] = (int32_t)first[t].key; }
    tile_first[T] = (int32_t)L;
    int64_t grp = -1;
    for (int64_t s = 0; s < L; ++s) {
        if (s == 0 || pr[s].key != pr[s - 1].key) ++grp;
        tile_of[pr[s].idx] = rank[grp];
    }
    /* halo of each tile: its boxes' list entries, sorted, duplicates dropped */
    int64_t *hcount = (int64_t *)calloc((size_t)(T > 0 ? T : 1), sizeof(int64_t));
    int32_t **hal = (int32_t **)calloc((size_t)(T > 0 ? T : 1), sizeof(int32_t *));
    int64_t *hlen = (int64_t *)calloc((size_t)(T > 0 ? T : 1), sizeof(int64_t));
    for (int64_t A = 0; A < L; ++A) hcount[tile_of[A]] += nbr_start[A + 1] - nbr_start[A];
    for (int64_t t = 0; t < T; ++t) hal[t] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(hcount[t] > 0 ? hcount[t] : 1));
    for (int64_t A = 0; A < L; ++A) {
        int64_t t = tile_of[A];
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) hal[t][hlen[t]++] = nbr_idx[e];
    }
    halo_start[0] = 0;
    seg_start[0] = 0;
    for (int64_t t = 0; t < T; ++t) {
        qsort(hal[t], (size_t)hlen[t], sizeof(int32_t), orc_cmp_i32);
        int64_t u = 0;
        for (int64_t h = 0; h < hlen[t]; ++h)
            if (h == 0 || hal[t][h] != hal[t][h - 1]) hal[t][u++] = hal[t][h];
        hlen[t] = u;
        int64_t rows = 0;
        for (int64_t h = 0; h < u; ++h) rows += leaf_start[hal[t][h] + 1] - leaf_start[hal[t][h]];
        halo_start[t + 1] = halo_start[t] + u;
        seg_start[t + 1] = seg_start[t] + rows;
    }
    int64_t H = halo_start[T];
    *halo_total = H;
    if (H <= cap && halo_idx && red_row) {
        for (int64_t t = 0; t < T; ++t)
            for (int64_t h = 0; h < hlen[t]; ++h) halo_idx[halo_start[t] + h] = hal[t][h];
        for (int64_t A = 0; A < L; ++A) {
            int64_t t = tile_of[A];
            for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
                /* rows of the halo boxes before B in the tile's segment */
                int64_t row = seg_start[t];
                for (int64_t h = 0; h < hlen[t] && hal[t][h] != nbr_idx[e]; ++h)
                    row += leaf_start[hal[t][h] + 1] - leaf_start[hal[t][h]];
                red_row[e] = row;
            }
        }
    }
    for (int64_t t = 0; t < T; ++t) free(hal[t]);
    free(hal); free(hlen); free(hcount); free(rank); free(first); free(tile_of); free(pr);
    return T;
}

/* ------------------------------------------------------------------------ */
/* Locality (Definition 1, Formulas (10)-(11))                              */
/* ------------------------------------------------------------------------ */

/* Dispersion of the gather layout: for each target leaf, the number of
 * maximal runs of consecutive leaf ids in its near list (leaves are stored
 * contiguously in id order, so a run is one contiguous memory block).  The
 * redundant layout reads one segment per leaf, D = 1.
 * out[0] = mean D (gather)      out[1] = V_gather = n * bytes_per_entry
 * out[2] = V_red = S * bytes    out[3] = D' = mean D / 1
 * out[4] = V' = V_gather/V_red  out[5] = Locality: D' V' if V_red <= C else V'/D' */
void orc_locality(int64_t L, const int64_t *nbr_start, const int32_t *nbr_idx, int64_t n,
                  int64_t S, double bytes_per_entry, double cache_bytes, double *out)
{
    double sumD = 0.0;
    for (int64_t A = 0; A < L; ++A) {
        int64_t runs = 0;
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e)
            if (e == nbr_start[A] || nbr_idx[e] != nbr_idx[e - 1] + 1) ++runs;
        sumD += (double)runs;
    }
    double Dbar = L > 0 ? sumD / (double)L : 0.0;
    double Vg = (double)n * bytes_per_entry, Vr = (double)S * bytes_per_entry;
    double Dp = Dbar / 1.0, Vp = Vr > 0 ? Vg / Vr : 0.0;
    out[0] = Dbar; out[1] = Vg; out[2] = Vr; out[3] = Dp; out[4] = Vp;
    out[5] = (Vr <= cache_bytes) ? Dp * Vp : (Dp > 0 ? Vp / Dp : 0.0);
}
