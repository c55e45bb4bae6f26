/*
 * p2p.h -- C ABI of libp2p, the MI355X (gfx950) near-field (P2P) operator of
 * the multilevel fast multipole algorithm, with the data-redundancy layout of
 * arXiv 2511.21535 ("Modeling the Effect of Data Redundancy on Speedup in
 * MLFMA Near-Field Computation").
 *
 * The operator (Sec. 1 and Sec. 2.1 of the paper): every target in a leaf box
 * interacts directly with every source in the leaf itself and in the leaf
 * boxes around it (the order-1-box stencil of Sec. 2.2, the E2 neighbourhood
 * of Sec. 5.1).  Two layouts feed the same sum:
 *   - GATHER: sources are read from the box-sorted arrays through the
 *     near-field lists (the paper's SoA + indexing baseline, Sec. 5.2.1);
 *   - REDUNDANT: each target box's near sources are first copied into one
 *     contiguous segment (the paper's data redundancy, Sec. 1.1, Sec. 5.2.1),
 *     a restructuring step timed on its own (Proposition 2, Eq. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller, unless it
 *    is documented as a host pointer.  The library never allocates or frees
 *    device memory: scratch space comes from `ws`.
 *  - Workspace protocol: call with ws == NULL to get the required size in
 *    *ws_bytes (returns P2P_OK and does nothing else); then call again with a
 *    device buffer of at least that many bytes, 256-byte aligned, and
 *    *ws_bytes set to its size.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream).  p2p_build_tree and p2p_build_neighbors read counts back to
 *    the host and therefore synchronise `stream`; p2p_restructure_redundant
 *    does so only when the near lists do not carry the layout size
 *    (nbrs->red_entries < 0); the evaluation and adjoint calls never do.
 *  - Validation happens on the host before any launch.  On P2P_EINVAL,
 *    P2P_EDOMAIN or P2P_ECAPACITY no output has been written (except the
 *    documented count fields).  On P2P_EHIP the outputs are undefined.
 *    Faults inside kernels surface at the next synchronising call.
 *  - p2p_last_error() describes the last failure on the calling thread.
 *  - Calls on different streams may run concurrently; calls that share a
 *    workspace buffer must not overlap.
 *  - HIP graphs: every evaluation, the adjoint and the restructures over near
 *    lists that carry their size only enqueue kernels and may be captured
 *    into a graph and replayed (with the same arrays and workspace).  Calls
 *    that read counts back, synchronise or copy from host memory -- building
 *    trees and near lists, p2p_locality, restructures over lists without
 *    their size, and Helmholtz evaluations that upload their parameters (more
 *    than 8 grid instances or G tables, several right-hand sides, FP64) --
 *    return P2P_EUNSUPPORTED while `stream` is capturing, before queueing
 *    anything.
 *
 * Readings of the paper (it gives no kernel formulas; these are the ones this
 * library adopts):
 *  - gravity: G = 1, Plummer softening, phi_i = -sum m_j (r^2+eps^2)^{-1/2},
 *    a_i = -sum m_j (x_i-x_j)(r^2+eps^2)^{-3/2}, the self pair j = i excluded;
 *  - Helmholtz: G(r) = e^{ikr}/(4 pi r) in 3-D, r = 0 excluded;
 *  - near field: leaves whose closed cubes touch, the leaf itself included;
 *    optionally (particle trees) on the unit torus, where a leaf's periodic
 *    images count as leaves of their own (the periodic interactions of the
 *    stellar-dynamics case, Sec. 5.2);
 *  - the redundancy grain is the target box.
 */
#ifndef P2P_H
#define P2P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *p2p_stream_t; /* hipStream_t */

typedef enum {
    P2P_OK = 0,
    P2P_EINVAL = 1,       /* bad argument (null pointer, negative size, bad mode, ws too small) */
    P2P_EDOMAIN = 2,      /* a particle coordinate outside [0,1) (or NaN) */
    P2P_ECAPACITY = 3,    /* an output capacity is too small; the count field holds the need */
    P2P_EHIP = 4,         /* a HIP runtime call failed */
    P2P_EUNSUPPORTED = 5  /* valid but not provided combination */
} p2p_status;

typedef enum { P2P_GATHER = 0, P2P_REDUNDANT = 1 } p2p_layout;

/* P2P_FP64: every operation in double precision.
 * P2P_FP32_MIXED: pair arithmetic in single precision; double precision only
 * for removing the large offset from coordinates (gravity: each position is
 * taken relative to the centre of the target leaf in double and rounded to
 * single once per (target leaf, source)) and for the per-target accumulation
 * of single-precision partial sums (gravity: at most 32 pair terms each;
 * Helmholtz: the 64 terms of one near box, each box's FP32 partial product
 * added into a double sum per target and right-hand side).  Helmholtz
 * blocks run on FP32 matrix cores when there is one right-hand side or a
 * multiple of 32.
 * P2P_FP32 (Helmholtz only; gravity calls return P2P_EUNSUPPORTED): as
 * FP32_MIXED, but the sums over all near boxes stay in single precision.
 * Layouts built with FP32_MIXED and FP32 hold the same payload and serve
 * either. */
typedef enum { P2P_FP64 = 0, P2P_FP32_MIXED = 1, P2P_FP32 = 2 } p2p_precision;

enum { P2P_TREE_PARTICLES = 0, P2P_TREE_GRIDS = 1 };
enum { P2P_KIND_GRAVITY = 0, P2P_KIND_HELMHOLTZ = 1 };

/* One regular-grid instance (host struct).  n_side^3 points, cell-centred at
 * ((i+0.5)h, (j+0.5)h, (k+0.5)h), caller index point_off + i + n(j + n k).
 * Instances are concatenated in caller order: point_off of instance g+1 is
 * point_off[g] + n_side[g]^3, and point_off[0] = 0. */
typedef struct {
    int32_t n_side;   /* multiple of 4, 4..1024 */
    int32_t reserved; /* must be 0 */
    double h;         /* spacing > 0 */
    double k;         /* wavenumber >= 0 */
    int64_t point_off;
} p2p_grid;

/* Octree (particles) or box grid (grids).  Host struct holding device
 * pointers.  Keys:
 *   particles: c_d = floor(x_d 2^20), key = Morton(c) (bit 3b of the key is
 *     bit b of c_x, 3b+1 of c_y, 3b+2 of c_z), 60 bits;
 *   grids: with b = smallest integer >= 2 such that 2^b >= max n_side,
 *     key = (g << 3b) | Morton_b(i, j, k).
 * perm lists caller indices sorted stably by (key, caller index).
 * Leaves (never empty) are in ascending key order; leaf_key is the key of the
 * leaf's lower corner, leaf_level its level (particles: a level-l leaf has
 * edge 2^-l; grids: b - 2, boxes of 4x4x4 points). */
typedef struct {
    int64_t n;           /* in: number of points */
    int64_t cap_leaves;  /* in: capacity of leaf_key/leaf_level (leaf_start: cap_leaves+1);
                            cap_leaves >= n always suffices */
    int64_t n_leaves;    /* out: L */
    int32_t kind;        /* out: P2P_TREE_PARTICLES or P2P_TREE_GRIDS */
    int32_t key_bits;    /* out: bits per axis of the key space (20, or b for grids) */
    int32_t max_level;   /* out: deepest leaf level */
    int32_t n_grids;     /* out: number of grid instances (0 for particles) */
    int32_t *perm;       /* device [n]: sorted slot -> caller index */
    int32_t *leaf_start; /* device [L+1]: first sorted slot of each leaf; leaf_start[L] = n */
    uint64_t *leaf_key;  /* device [L] */
    int8_t *leaf_level;  /* device [L] */
    int32_t *iperm;      /* device [n]: caller index -> sorted slot (the inverse of perm) */
} p2p_tree;

/* Near-field lists in CSR form: nbr(A) = nbr_idx[nbr_start[A] .. nbr_start[A+1]),
 * every leaf whose closed cube touches A's (same grid instance), A included,
 * ascending.
 * Periodic lists (periodic = 1, particle trees only): the domain [0,1)^3 is a
 * torus.  An entry is a leaf B together with an image code
 * c = (sx+1) + 3 (sy+1) + 9 (sz+1), sx, sy, sz in {-1, 0, 1}, in
 * nbr_shift[e]: B's points taken at x + (sx, sy, sz), B's cube shifted the
 * same way touching A's.  Code 13 is the unshifted leaf.  Entries are in
 * ascending (c, B); one leaf can appear under several codes (a leaf touching
 * A across a face of the domain and inside it), and the self pair skipped by
 * the sums is only the point itself in the unshifted image.  The relation is
 * symmetric: (B, c) in nbr(A) iff (A, 26 - c) in nbr(B). */
typedef struct {
    int64_t cap;         /* in: capacity of nbr_idx (and nbr_shift) */
    int64_t count;       /* out: E = total entries (also on P2P_ECAPACITY) */
    int64_t *nbr_start;  /* device [L+1] */
    int32_t *nbr_idx;    /* device [cap] */
    int64_t red_entries; /* out: S = sum over A of the points of the leaves in
                            nbr(A), the size of the redundant layout over these
                            lists; a caller that fills the lists itself sets -1
                            (unknown) */
    int32_t periodic;    /* in: 0 = plain lists, 1 = periodic images (above) */
    int32_t reserved;    /* must be 0 */
    int8_t *nbr_shift;   /* device [cap]: image code per entry; used only when
                            periodic = 1 (then required once E > 0) */
} p2p_nbrs;

/* Redundant layout.
 * Box grain (grain 0 or 1; the per-target redundancy of Sec. 5.2.1):
 * segment A = entries [red_start[A], red_start[A+1]) holds, for B in nbr(A)
 * in order, the rows of B's sorted slots in order; A's own rows (the
 * unshifted image) start at red_start[A] + red_self[A].  S = red_start[L]
 * entries.  With periodic lists the gravity rows of an entry hold the shifted
 * positions x + s.
 * Tile grain (grain 2 or 4, grid trees only; the per-block redundancy that
 * Sec. 3.5 names for dense regular distributions): the boxes of an instance
 * are grouped into tiles, aligned blocks of grain^3 boxes (fewer at the upper
 * faces), each one contiguous run of leaves in key order.  A tile's segment
 * holds the rows of its halo -- the union of its boxes' near lists -- box by
 * box in ascending leaf id, 64 rows per box; tiles follow each other in leaf
 * order.  red_start[A] is the first row of the segment of A's tile (so
 * red_start[L] = S), and red_row[e], for entry e = (A, B) of the near lists,
 * the first row of B in that segment.  red_self is not written.  A box's
 * sources are read through red_row; the layout holds about
 * ((grain+2)/grain)^3 copies of each box instead of 27.
 * Payload planes (device):
 *   gravity FP64: planes[0] = double[S][4] rows (x, y, z, m), 32-byte rows;
 *   gravity FP32_MIXED: planes[0] = float4[S] (x - c, y - c, z - c, m), where c
 *     is the centre of the segment's target leaf, the difference taken in
 *     double and rounded to float once (the large offset removed in double,
 *     so pair differences are float differences of small numbers);
 *     planes[1..3] unused;
 *   Helmholtz: planes[0] = q rows, [S][nrhs] complex (float2 for FP32_MIXED,
 *     double2 for FP64); planes[1..3] unused. */
typedef struct {
    int64_t cap;        /* in: capacity in entries of every plane */
    int64_t count;      /* out: S (also on P2P_ECAPACITY) */
    int64_t *red_start; /* device [L+1] */
    int32_t *red_self;  /* device [L] */
    void *planes[4];
    int32_t nrhs;       /* out: RHS per row (Helmholtz) */
    int32_t kind;       /* out: P2P_KIND_* */
    int32_t prec;       /* out: p2p_precision of the payload */
    int32_t grain;      /* in: 0 or 1 = box grain; 2 or 4 = tiles of grain^3 boxes (grid trees) */
    int64_t *red_row;   /* device [E] (tile grain): first row of each near-list entry's source box */
} p2p_redundant;

/* Per-interaction redundant layout (gravity; the thread-level redundancy of
 * the paper's stellar-dynamics case, Sec. 5.2.1, whose data volumes Table 5
 * compares): one record per near-list entry e = (A, B) in CSR order, rows
 * [rec_start[e], rec_start[e+1]): a header row holding occ_A, occ_B, A and B
 * as integers (int32 bit patterns in the four floats of an FP32_MIXED row,
 * exact integers in the four doubles of an FP64 row), then the occ_A rows of
 * A's points (the targets), then the occ_B rows of B's points (the sources),
 * each in sorted order, with the payload of the box-grain layout (FP32_MIXED:
 * float4 (x - c_A, y - c_A, z - c_A, m) relative to the centre of A; FP64:
 * double[4] (x, y, z, m); with periodic lists B's rows hold the shifted
 * positions x + s).  Every record can be evaluated on its own (the evaluation
 * reads the entry's image code only to tell the self record (A, A, 13)); the
 * results of the records of one target leaf are then summed (the update). */
typedef struct {
    int64_t cap;        /* in: capacity in rows of planes[0] */
    int64_t count;      /* out: rows = E + sum_e (occ_A + occ_B) (also on P2P_ECAPACITY) */
    int64_t *rec_start; /* device [E+1] */
    void *planes[1];    /* device rows: float4 (FP32_MIXED) or double[4] (FP64) */
    int64_t target_rows;/* out: sum_e occ_A, the result rows the evaluation needs */
    int32_t prec;       /* out: p2p_precision of the payload */
    int32_t reserved;
} p2p_interactions;

/* Locality metric (Definition 1, Formulas (10)-(11) of the paper). */
typedef struct {
    double d_mean;       /* mean over target leaves of D = runs of consecutive ids in nbr(A) */
    double v_gather;     /* bytes of the gather layout: n * bytes_per_entry */
    double v_red;        /* bytes of the redundant layout: S * bytes_per_entry */
    double d_ratio;      /* D' = d_mean / 1 (the redundant layout has D = 1) */
    double v_ratio;      /* V' = v_gather / v_red */
    double locality;     /* D' V' if v_red <= cache_bytes (10), else V'/D' (11) */
    int64_t pairs;       /* ordered near pairs, self excluded */
    int64_t entries;     /* S */
} p2p_locality_t;

/* Build the tree (binning; the stellar-dynamics code of Sec. 4 rebuilds it
 * every time step, and Sec. 1.1 names tree building, the data collection, a
 * major overhead).
 *  Particles: x, y, z caller-order double[n] in [0,1) (else P2P_EDOMAIN),
 *    grids == NULL, n_grids == 0.  leaf_cap == 0: uniform tree of depth
 *    `depth` (0..20, empty leaves dropped).  leaf_cap > 0: adaptive tree, a
 *    node splits iff it holds more than leaf_cap points and its level is
 *    below `depth` (1..20).
 *  Grids: x = y = z = NULL, grids = host array of n_grids instances,
 *    tree->n = total points; depth and leaf_cap ignored.
 * tree->perm and tree->iperm must hold n entries each, the leaf arrays
 * cap_leaves (+1).  Synchronises `stream` (reads L back).  P2P_ECAPACITY if
 * L > cap_leaves (tree->n_leaves holds L). */
p2p_status p2p_build_tree(const double *x, const double *y, const double *z,
                          const p2p_grid *grids, int32_t n_grids,
                          int32_t depth, int32_t leaf_cap,
                          p2p_tree *tree, void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Near-field lists of every leaf (the E2 neighbourhood, Sec. 5.1;
 * Fig. 8 counts them for irregular trees).  nbrs->nbr_start must hold L+1
 * entries; nbrs->periodic selects periodic images (P2P_EINVAL on a grid
 * tree), which also fills nbrs->nbr_shift.  Also sets nbrs->red_entries.
 * Synchronises `stream`; P2P_ECAPACITY if E > nbrs->cap (count and
 * red_entries are still set). */
p2p_status p2p_build_neighbors(const p2p_tree *tree, p2p_nbrs *nbrs,
                               void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Restructure to the redundant layout (data redundancy, Sec. 1.1 and
 * Sec. 5.2.1; its cost is the "collect" term of Eq. 2).
 *  Gravity trees (particles): src = {x, y, z, m} caller-order double[n];
 *    the payload follows `prec` (FP32_MIXED stores m rounded to float).
 *  Helmholtz trees (grids): src[0] = q caller-order [n][nrhs] complex
 *    (float2 for FP32_MIXED, double2 for FP64), src[1..3] ignored.
 * out->red_start (L+1), out->red_self (L) and the planes must be allocated;
 * P2P_ECAPACITY (out->count = S) if S > out->cap.  S is taken from
 * nbrs->red_entries; only if that is negative is it counted on the GPU and
 * read back (synchronising `stream`).
 * out->grain selects the redundancy grain (see p2p_redundant): 0 or 1 box
 * grain; 2 or 4 tiles (grid trees only, else P2P_EINVAL), which needs
 * out->red_row (nbrs->count entries); the tile layout's size is counted on
 * the GPU and read back (synchronising `stream`), and its rows are read from
 * q through tree->perm (no sorted copy). */
p2p_status p2p_restructure_redundant(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                     const void *const src[4], int32_t nrhs,
                                     p2p_precision prec, p2p_redundant *out,
                                     void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Near-field gravity (the P2P compute step of Eq. 2, Sec. 3.2, from the
 * GATHER layout -- the SoA + indexing baseline of Sec. 5.2.1 -- or from the
 * REDUNDANT layout of Sec. 5.2.1; the update step of Eq. 2 fused): for every
 * particle i, phi_i and a_i as in the header comment, eps >= 0 (eps == 0
 * drops pairs at zero distance and needs distinct points at least 2^-511
 * apart in FP64, whose r^-1 is formed for r^2 >= 2^-1022; a positive eps must be >= 1e-4 with
 * FP32_MIXED, whose add-back of the target's own term m_i/eps leaves its
 * float rounding in phi_i, and >= 2^-511 with FP64, which drops that pair by
 * position; smaller positive eps is P2P_EINVAL).  x, y, z, m: caller-order double[n] (needed
 * for GATHER; ignored for REDUNDANT, which reads `red`, built with the same
 * precision).  Outputs phi, ax, ay, az: caller-order double[n], overwritten. */
p2p_status p2p_eval_gravity(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                            p2p_layout layout, p2p_precision prec, double eps,
                            const double *x, const double *y, const double *z, const double *m,
                            double *phi, double *ax, double *ay, double *az,
                            void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as p2p_eval_gravity, same arguments and results, without a
 * workspace.  The GATHER layout's box-sorted rows go to a static scratch array
 * inside the library, 2^21 rows of 32 bytes (64 MiB), one copy per GPU, held
 * until the process ends; REDUNDANT needs no scratch.  tree->n above 2^21 with
 * GATHER returns P2P_EUNSUPPORTED before anything is queued.  Calls on one GPU
 * share that GPU's scratch: two calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and give undefined
 * results; calls ordered on one stream are safe.  Every scratch row that is
 * read is first written by the same call.  Allocates nothing. */
p2p_status p2p_eval_gravity_noalloc(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                                    p2p_layout layout, p2p_precision prec, double eps,
                                    const double *x, const double *y, const double *z, const double *m,
                                    double *phi, double *ax, double *ay, double *az,
                                    p2p_stream_t stream);

/* Near-field Helmholtz on grid trees (the dense regular case of Sec. 5.1, the
 * near-field part of the MLFMA call of Sec. 4-5.1, with precomputed
 * interaction patterns; single RHS, multi-RHS, and many instances in one
 * batched persistent launch): u_I = sum_{J near I, J != I} e^{ik r}/(4 pi r) q_J
 * for each of the nrhs columns, with h and k of I's instance.  grids: the host
 * array the tree was built from.  q (GATHER) and u: caller order [n][nrhs],
 * float2 (FP32_MIXED) or double2 (FP64) interleaved complex.  REDUNDANT reads
 * q from `red` (built with the same precision and nrhs).  FP32_MIXED with
 * nrhs a multiple of 32 (at most 2^20) runs on FP32 matrix cores (v_mfma_f32_32x32x2f32) in
 * one persistent launch over all boxes of all instances, taking (box, RHS
 * chunk) items in tree order from eight queues, one per XCD, each over a
 * contiguous eighth of the items, a wave whose own queue is empty taking from
 * the others in turn (neighbouring boxes meet in one XCD's L2); instances whose k h
 * agree to 1e-12 share one set of G blocks.  nrhs == 1 runs on the matrix
 * cores of its precision (v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64) with
 * tiles of 16 target boxes as the columns of the product.  `tile` (host int32[4], may be
 * NULL = default {4, 2, 64 or 32, 1}) is the launch shape the autotuner picked:
 * tile[0] = waves per workgroup (1, 2 or 4), tile[1] = workgroups per compute
 * unit (1..16), tile[2] = right-hand sides per wave (32 or 64, dividing nrhs),
 * tile[3] = copies of the G blocks in memory (1, 2, 4 or 8; the block-level
 * pattern redundancy factor of Sec. 5.1.2, the workgroups of one XCD reading
 * different copies); other paths reject a non-NULL tile with P2P_EINVAL. */
p2p_status p2p_eval_helmholtz(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                              p2p_layout layout, p2p_precision prec,
                              const p2p_grid *grids, int32_t n_grids, int32_t nrhs,
                              const void *q, void *u, const int32_t *tile,
                              void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Precomputed interaction patterns for the Helmholtz evaluation (the dense
 * regular case of Sec. 5.1, where the near-field patterns are computed once and
 * reused by every box and every call).  A plan holds, in a caller-owned device
 * buffer, what p2p_eval_helmholtz otherwise rebuilds on every call: the
 * instances' parameters, the G blocks of every distinct k h built in double
 * precision (rounded to single on the FP32 matrix-core paths) or the G(d^2)
 * tables (vector path).  Host struct. */
typedef struct {
    void *buf;            /* in: device buffer, 256-byte aligned; NULL asks for the size */
    size_t bytes;         /* in: size of buf; out (buf == NULL): bytes needed */
    int32_t prec;         /* out: p2p_precision the plan serves */
    int32_t nrhs;         /* out: right-hand sides per call */
    int32_t tile[4];      /* out: launch shape (as for p2p_eval_helmholtz) */
    int32_t tiled;        /* out: 1 if a tile was given to p2p_helmholtz_prepare */
    int32_t reserved;
    uint64_t fingerprint; /* out: of the sizes of tree and lists, the grids, prec,
                             nrhs and tile; 0 = not prepared */
} p2p_helmholtz_plan;

/* Build a plan for evaluations on `tree`/`nbrs` with these grids, precision,
 * nrhs and tile (arguments as for p2p_eval_helmholtz).  With plan->buf ==
 * NULL only plan->bytes is written.  Otherwise the set-up is queued on
 * `stream` into plan->buf (P2P_EINVAL if plan->bytes is too small).  Plans
 * whose parameters do not travel in the kernel arguments (more than 8
 * instances or G tables, several right-hand sides, FP64) copy them from host
 * memory: P2P_EUNSUPPORTED while `stream` is capturing.  The plan stays
 * valid while the tree, the lists and the grids stay as they were. */
p2p_status p2p_helmholtz_prepare(const p2p_tree *tree, const p2p_nbrs *nbrs, p2p_precision prec,
                                 const p2p_grid *grids, int32_t n_grids, int32_t nrhs,
                                 const int32_t *tile, p2p_helmholtz_plan *plan, p2p_stream_t stream);

/* p2p_eval_helmholtz from a plan: the same results, with the precision, nrhs
 * and tile of the plan, and no set-up work: a REDUNDANT call is one product
 * launch (two with several right-hand sides: the work-queue counters are
 * zeroed first), a GATHER call adds the copy of q into box order.  The
 * workspace holds only that copy and the counters.  P2P_EINVAL if the plan was
 * prepared for other sizes, grids, precision, nrhs or tile.  Never copies
 * from host memory or synchronises, so it may be captured into a HIP graph.
 * Calls that share one plan may overlap (the plan is only read). */
p2p_status p2p_eval_helmholtz_prepared(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                                       p2p_layout layout, const p2p_grid *grids, int32_t n_grids,
                                       const p2p_helmholtz_plan *plan, const void *q, void *u,
                                       void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Adjoint (not in the paper; the gradient that the DBIM inversion of Sec. 4
 * descends along, and the stellar-dynamics forces differentiated).
 *  kind == P2P_KIND_GRAVITY: fwd_in = {x, y, z, m}, grad_out = {g_phi, g_ax,
 *    g_ay, g_az}, grad_in = {g_x, g_y, g_z, g_m}, all caller-order double[n]:
 *    the gradients of L = sum_i g_phi_i phi_i + g_a_i . a_i with respect to
 *    positions and masses (tree frozen), eps > 0 (FP64: eps >= 2^-511;
 *    FP32_MIXED: eps >= 1e-3, since the float rounding of the w^5 terms of
 *    close pairs grows as eps shrinks; else P2P_EINVAL).  GATHER layout; FP64, or
 *    FP32_MIXED (positions relative to the target leaf's centre, float pair
 *    terms, double accumulation, as in the forward evaluation).
 *  kind == P2P_KIND_HELMHOLTZ: grad_out[0] = g (caller order [n][nrhs]
 *    complex), grad_in[0] = A^T g, or conj(A^T conj(g)) = A^H g when
 *    `conjugate` is 1 (PyTorch's convention for complex gradients).  The
 *    near-field Helmholtz matrix is symmetric (reciprocity G(x,y) = G(y,x)
 *    and a symmetric near relation), so A^T = A.  grids/n_grids as for
 *    p2p_eval_helmholtz; fwd_in ignored. */
p2p_status p2p_adjoint(int32_t kind, const p2p_tree *tree, const p2p_nbrs *nbrs,
                       const p2p_redundant *red, p2p_layout layout, p2p_precision prec,
                       double eps, const p2p_grid *grids, int32_t n_grids, int32_t nrhs,
                       int32_t conjugate,
                       const void *const fwd_in[4], const void *const grad_out[4],
                       void *const grad_in[4], void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Restructure to the per-interaction layout (gravity trees only): src = {x, y,
 * z, m} caller-order double[n].  out->rec_start must hold E+1 entries.  The
 * row count is E + 2 S for lists built by p2p_build_neighbors (the near
 * relation is symmetric, so the targets of all records are S rows too);
 * otherwise it is counted on the GPU and read back (synchronising `stream`).
 * P2P_ECAPACITY (out->count = rows) if rows > out->cap. */
p2p_status p2p_restructure_interactions(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                        const double *const src[4], p2p_precision prec,
                                        p2p_interactions *out, void *ws, size_t *ws_bytes,
                                        p2p_stream_t stream);

/* Near-field gravity from the per-interaction layout: every record's pair sums
 * (phi, a as in the header comment, eps >= 0, the precision of `inter`) go to
 * result rows of their own in the workspace (target_rows x 32 bytes), then
 * each target's results over the records of its leaf are summed in FP64 and
 * written to phi, ax, ay, az (caller-order double[n], overwritten). */
p2p_status p2p_eval_gravity_interactions(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                         const p2p_interactions *inter, double eps,
                                         double *phi, double *ax, double *ay, double *az,
                                         void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Remote interactions (the remote type of the stellar-dynamics case, Sec. 5.2,
 * computed in its own launch beside the local and periodic ones: targets of
 * this domain, sources received from another).  `tree` holds the targets,
 * `src_tree` the sources, another particle set in the same unit cube with its
 * own tree; both are particle trees and distinct structures.  The lists of
 * p2p_build_neighbors_remote are CSR over the leaves of `tree` (nbr_start has
 * L+1 entries) with entries that index the leaves of `src_tree`: every source
 * leaf whose closed cube touches the target leaf, ascending, through the
 * periodic images when nbrs->periodic (codes and order as for periodic plain
 * lists).  A list may be empty.  red_entries counts the source points in the
 * lists.  Synchronises `stream`; P2P_ECAPACITY as p2p_build_neighbors. */
p2p_status p2p_build_neighbors_remote(const p2p_tree *tree, const p2p_tree *src_tree, p2p_nbrs *nbrs,
                                      void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Redundant layout of the remote sources: as p2p_restructure_redundant for
 * gravity, the segment of target leaf A holding the rows of the source points
 * of the leaves in its remote list (src = the source set's caller-order x, y,
 * z, m; FP32_MIXED rows relative to the centre of A).  red_self is -1 (the
 * targets are not among the sources).  Synchronises `stream` only when
 * nbrs->red_entries < 0. */
p2p_status p2p_restructure_remote(const p2p_tree *tree, const p2p_tree *src_tree, const p2p_nbrs *nbrs,
                                  const double *const src[4], p2p_precision prec, p2p_redundant *out,
                                  void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Remote gravity: for every target point i, the sums of the header comment
 * over the source points j of its leaf's remote list (each at its image), no
 * pair skipped (the two sets are distinct; eps == 0 drops pairs at zero
 * distance), ADDED to phi, ax, ay, az (caller order of the targets), so that a
 * remote call after the local one completes the near field.  x, y, z: the
 * targets' caller-order positions (always read); sx, sy, sz, sm: the
 * sources' (GATHER; REDUNDANT reads `red`, built by p2p_restructure_remote
 * with the same precision). */
p2p_status p2p_eval_gravity_remote(const p2p_tree *tree, const p2p_tree *src_tree, const p2p_nbrs *nbrs,
                                   const p2p_redundant *red, p2p_layout layout, p2p_precision prec,
                                   double eps, const double *x, const double *y, const double *z,
                                   const double *sx, const double *sy, const double *sz, const double *sm,
                                   double *phi, double *ax, double *ay, double *az,
                                   void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Locality metric per configuration (Definition 1 and Formulas (10)-(11),
 * Sec. 3.4).  D per target leaf is counted on the GPU from the near lists;
 * the rest is host arithmetic.  red may be NULL (S is then computed from the
 * lists).  Synchronises `stream`. */
p2p_status p2p_locality(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                        double bytes_per_entry, double cache_bytes, p2p_locality_t *out,
                        void *ws, size_t *ws_bytes, p2p_stream_t stream);

/* Description of the last failure on the calling thread; valid until the
 * next p2p_* call on that thread.  Never NULL. */
const char *p2p_last_error(void);

/* Library version string. */
const char *p2p_version(void);

#ifdef __cplusplus
}
#endif
#endif /* P2P_H */
