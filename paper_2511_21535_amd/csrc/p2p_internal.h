// Internal declarations shared by the libp2p translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "p2p.h"

namespace p2p {

// One particle row (x, y, z, m) or four gradient components, 32-byte aligned so
// a row moves as two 16-byte accesses.
struct alignas(32) Row4d {
    double x, y, z, w;
};

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
p2p_status fail(p2p_status st, const std::string &msg);

#define P2P_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::p2p::fail(P2P_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define P2P_LAUNCH_CHECK()                                                                 \
    do {                                                                                   \
        hipError_t e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess)                                                              \
            return ::p2p::fail(P2P_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

#define P2P_TRY(expr)                                                                      \
    do {                                                                                   \
        p2p_status s_ = (expr);                                                            \
        if (s_ != P2P_OK) return s_;                                                       \
    } while (0)

// ------------------------------------------------------------- workspace --
// Carves 256-byte aligned sub-buffers out of one caller buffer.  With a null
// base it only measures.
struct Arena {
    char *base;
    size_t used = 0;
    explicit Arena(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T) + 256;
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

// -------------------------------------------------------------- launches --
inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

// Device scan: exclusive prefix sum of in[0..n) into out[0..n], out[n] = total.
// In-place allowed.  Scratch from scan_ws_elems(n) elements of type TO.
size_t scan_ws_elems(int64_t n);
template <class TI, class TO>
p2p_status exclusive_scan(const TI *in, TO *out, int64_t n, TO *scratch, hipStream_t s);

// Sort (key, value) pairs by key, stably, over the low `key_bits` bits.
// keys/vals are sorted in place; tmp buffers of the same sizes are needed.
p2p_status radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp,
                            int64_t n, int key_bits, uint32_t *hist_scratch, hipStream_t s);
size_t radix_hist_elems(int64_t n);

// Tree construction steps (tree.hip).
p2p_status launch_particle_keys(const double *x, const double *y, const double *z, int64_t n,
                                uint64_t *keys, int32_t *vals, int32_t *bad_flag, hipStream_t s);
p2p_status launch_grid_keys(const int32_t *d_n_side, const int64_t *d_point_off, int32_t n_grids,
                            int bits, int64_t n, uint64_t *keys, int32_t *vals, hipStream_t s);
p2p_status launch_leaf_levels(const uint64_t *skeys, int64_t n, int kind, int depth, int leaf_cap,
                              uint8_t *pair_common, int8_t *level, int32_t *flags, hipStream_t s);
p2p_status launch_perm_and_inverse(const int32_t *vals, int64_t n, int32_t *perm, int32_t *iperm,
                                   hipStream_t s);
// Leaf arrays from the start flags and their scan, then the deepest level into
// *max_level.
p2p_status launch_leaf_write(const uint64_t *skeys, const int8_t *level, const int32_t *flags,
                             const int32_t *flag_scan, int64_t n, int kind, int32_t *leaf_start,
                             uint64_t *leaf_key, int8_t *leaf_level, int32_t *max_level,
                             hipStream_t s);

// Near lists (nbrs.hip).  Directory over the top bits of the leaf keys (dir:
// (1 << neighbor_dir_bits) + 1 entries); it also clears the overflow counter.
int neighbor_dir_bits(int total_key_bits);
// counters[2]: lists over kNbrSlotsPerLeaf entries, heavy leaves (cleared here).
p2p_status launch_key_directory(const uint64_t *leaf_key, int64_t L, int total_key_bits, int32_t *dir,
                                int32_t *counters, hipStream_t s);
// Near lists in two passes.  The counting pass writes per-leaf counts, segment
// lengths (points of the leaves in the list) and the first 64 entries of each
// list into slots[L][64]; after the scan of the counts, the fill moves the
// slots into the CSR and searches again only for the lists longer than 64.
// Leaves with many candidates are listed in heavy[L] and searched by a whole
// workgroup each.  With tg set, the lists belong to tg's leaves (counts, segs,
// slots, heavy, nbr_start sized by tg->L) and the candidates are the leaves of
// the tree passed as leaf_key/leaf_level/leaf_start/L (remote lists).
struct NbrTargets {
    const uint64_t *leaf_key;
    const int8_t *leaf_level;
    int64_t L;
};
// A non-null slot_code selects periodic lists (particles on the unit torus):
// slot_code[L][64] and nbr_shift then receive the image codes.
constexpr int kNbrSlotsPerLeaf = 64;
p2p_status launch_neighbors_count(const uint64_t *leaf_key, const int8_t *leaf_level, int64_t L,
                                  int key_bits, int inst_shift, const int32_t *dir, int total_key_bits,
                                  const int32_t *leaf_start, int32_t *counts, int32_t *segs,
                                  int32_t *slots, int8_t *slot_code, int32_t *counters, int32_t *heavy,
                                  hipStream_t s, const NbrTargets *tg = nullptr);
p2p_status launch_nbr_totals(const int64_t *start, const int64_t *seg_scan, const int32_t *counters,
                             int64_t L, int64_t *out, hipStream_t s);
p2p_status launch_neighbors_fill(const uint64_t *leaf_key, const int8_t *leaf_level, int64_t L,
                                 int key_bits, int inst_shift, const int32_t *dir, int total_key_bits,
                                 const int32_t *counts, const int32_t *slots, const int8_t *slot_code,
                                 int32_t *counters, const int32_t *heavy, bool any_overflow,
                                 const int64_t *nbr_start, int32_t *nbr_idx, int8_t *nbr_shift, hipStream_t s,
                                 const NbrTargets *tg = nullptr);

// Restructure (restructure.hip).
// Segment lengths of L target leaves over the source leaves of leaf_start.
// nbr_shift (image codes, may be null) places the unshifted self image; with
// self_in_list false (remote lists) red_self is -1.
p2p_status launch_seg_lengths(const int32_t *leaf_start, const int64_t *nbr_start,
                              const int32_t *nbr_idx, const int8_t *nbr_shift, int64_t L,
                              int32_t *seg_len, int32_t *red_self, bool self_in_list, hipStream_t s);
template <class T>
p2p_status launch_permute_rows(const T *src, const int32_t *perm, int64_t n, int64_t row_len,
                               T *dst, hipStream_t s);
// Caller-order planes (a, b, c, d) into sorted rows: out[iperm[i]] = (a, b, c, d)[i].
p2p_status launch_scatter4(const double *a, const double *b, const double *c, const double *d,
                           const int32_t *iperm, int64_t n, Row4d *out, hipStream_t s);
// Gravity payload from sorted rows: FP64 rows (d8) or, for FP32_MIXED, float4
// (x - c_A, y - c_A, z - c_A, m) relative to the centre of target leaf A (d4).
// With image codes (nbr_shift not null) each source is placed at x + s.
// With pr set, the source rows are read through pr->perm (sorted slot -> caller
// index) from the caller-order planes pr->x, y, z, m instead of `sorted`.
struct PermRows {
    const double *x, *y, *z, *m;
    const int32_t *perm;
};
p2p_status launch_copy_segments_gravity(const Row4d *sorted, const uint64_t *leaf_key,
                                        const int8_t *leaf_level, const int32_t *leaf_start,
                                        const int64_t *nbr_start, const int32_t *nbr_idx,
                                        const int8_t *nbr_shift, const int64_t *red_start, int64_t L,
                                        Row4d *d8, float4 *d4, bool streaming, hipStream_t s,
                                        const PermRows *pr = nullptr);
// Segment offsets of layouts whose leaves all hold box_rows points (grid
// boxes): red_start[A] = box_rows nbr_start[A] and red_self[A] = box_rows
// times A's place in its list, written by the copy itself (box_rows = 0: the
// copy reads red_start computed beforehand).
struct BoxSegments {
    int64_t *red_start = nullptr;
    int32_t *red_self = nullptr;
    int32_t box_rows = 0;
    int64_t entries = 0;   // near-list entries (with box_rows > 0)
};
template <class T>
p2p_status launch_copy_segments(const T *sorted, int64_t row_len, const int32_t *leaf_start,
                                const int64_t *nbr_start, const int32_t *nbr_idx,
                                const int64_t *red_start, int64_t L, T *dst, bool streaming,
                                hipStream_t s, BoxSegments boxes = {});
// Tile grain on grid trees (restructure.hip).  Without hs: cnt[A] = halo size
// (boxes) of the tile whose first leaf is A, 0 for other leaves.  With hs (the
// exclusive scan of cnt, hs[L] = H): the halo lists into halo_idx, red_row for
// every near-list entry, red_start for every leaf and red_start[L].
p2p_status launch_tile_halo(const uint64_t *leaf_key, const int64_t *nbr_start, const int32_t *nbr_idx,
                            int64_t L, int key_bits, int grain, int64_t *cnt, const int64_t *hs,
                            int32_t *halo_idx, int64_t *red_row, int64_t *red_start, hipStream_t s);
// The tile segments: halo box j's 64 rows (caller rows of row_bytes each, read
// through perm) to rows [64 j, 64 j + 64) of dst.
p2p_status launch_tile_copy(const void *q, int64_t row_bytes, const int32_t *leaf_start, const int32_t *perm,
                            const int32_t *halo_idx, int64_t H, void *dst, bool streaming, hipStream_t s);
// Redundant layouts larger than this are written with streaming (nontemporal)
// stores; smaller ones stay in the 256 MB last-level cache for the evaluation.
constexpr int64_t kStreamingLayoutBytes = int64_t(128) << 20;

// Per-interaction layout (interactions.hip): one record per near-list entry e = (A, B),
// a header row (occ_A, occ_B, A, B as integers) then A's rows then B's rows,
// FP32_MIXED float4 relative to the centre of A, or FP64 rows; with image codes
// (nbr_shift not null) B's rows sit at x + s.
p2p_status launch_record_lengths(const int32_t *leaf_start, const int64_t *nbr_start,
                                 const int32_t *nbr_idx, int64_t L, int32_t *rec_len, int32_t *tgt_len,
                                 hipStream_t s);
p2p_status launch_copy_records(const Row4d *sorted, const uint64_t *leaf_key, const int8_t *leaf_level,
                               const int32_t *leaf_start, const int64_t *nbr_start,
                               const int32_t *nbr_idx, const int8_t *nbr_shift, const int64_t *rec_start,
                               int64_t L, Row4d *d8, float4 *d4, bool streaming, hipStream_t s);
// Pair sums of every record into its own result rows res[res_start[e] + t]
// (phi, ax, ay, az per target, FP64), then the per-target sums over the
// records of its leaf, written to caller order.  The self record is (A, A)
// in the unshifted image (nbr_shift null or code 13).
p2p_status launch_eval_records(const int64_t *rec_start, const Row4d *r8, const float4 *r4,
                               const int8_t *nbr_shift, int64_t E, const int64_t *res_start, double eps2,
                               bool eps_zero, Row4d *res, hipStream_t s);
p2p_status launch_reduce_records(const int32_t *leaf_start, const int64_t *nbr_start,
                                 const int64_t *res_start, const int32_t *perm, int64_t L,
                                 const Row4d *res, double *phi, double *ax, double *ay, double *az,
                                 hipStream_t s);

// Gravity (gravity.hip).
struct GravityArgs {
    int64_t L;
    const int32_t *leaf_start;
    const int32_t *perm;
    const uint64_t *leaf_key;
    const int8_t *leaf_level;
    const int64_t *nbr_start;
    const int32_t *nbr_idx;
    const int8_t *nbr_shift;          // image codes of periodic lists (gather), else null
    const int32_t *src_leaf_start;    // leaf starts of the source tree (leaf_start unless remote)
    const double *tx, *ty, *tz;       // remote: the targets' caller-order positions
    const double *sx, *sy, *sz, *sm;  // remote gather: the sources' caller-order arrays
    const int32_t *src_perm;          // remote gather: the source tree's perm
    const int64_t *red_start;
    const int32_t *red_self;
    const Row4d *s4;                  // FP64 rows (x, y, z, m): sorted (gather) or redundant (FP64)
    const float4 *red4;               // FP32_MIXED redundant payload (leaf-relative x, y, z, m)
    double eps2;
    double *phi, *ax, *ay, *az;       // caller order
};
p2p_status launch_gravity(const GravityArgs &a, bool redundant, bool mixed, bool eps_zero,
                          hipStream_t s);
// The evaluation behind p2p_eval_gravity (api.hip), split at the workspace:
// the argument checks that come before the workspace query, then the checks
// of the arrays and the launches, with the GATHER layout's sorted rows in s4
// (tree->n rows; unused for REDUNDANT).
p2p_status gravity_check_args(const p2p_tree *tree, const p2p_nbrs *nbrs, p2p_layout layout,
                              p2p_precision prec, double eps);
p2p_status gravity_run(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                       p2p_layout layout, p2p_precision prec, double eps, const double *x,
                       const double *y, const double *z, const double *m, double *phi, double *ax,
                       double *ay, double *az, Row4d *s4, hipStream_t s);
// Remote lists: targets read through perm from a.tx/ty/tz, sources of the
// source tree (gather: through a.src_perm from a.sx/sy/sz/sm; redundant: the
// remote segments), leaves with an empty list skipped, no self pair, sums
// added to phi, ax, ay, az.
p2p_status launch_gravity_remote(const GravityArgs &a, bool redundant, bool mixed, bool eps_zero,
                                 hipStream_t s);

struct GravityAdjointArgs {
    int64_t L;
    const int32_t *leaf_start;
    const int32_t *perm;
    const int64_t *nbr_start;
    const int32_t *nbr_idx;
    const int8_t *nbr_shift;                // image codes of periodic lists, else null
    const Row4d *s4;                        // sorted rows (x, y, z, m)
    const Row4d *g4;                        // sorted upstream gradients (g_phi, g_ax, g_ay, g_az)
    const uint64_t *leaf_key;               // FP32-mixed: the target leaf's centre
    const int8_t *leaf_level;
    double eps2;
    double *gx, *gy, *gz, *gm;              // caller order
};
p2p_status launch_gravity_adjoint(const GravityAdjointArgs &a, bool mixed, hipStream_t s);

// Helmholtz (helmholtz.hip).
struct HelmholtzArgs {
    int64_t L;
    int key_bits;
    const int32_t *leaf_start;
    const uint64_t *leaf_key;
    const int32_t *perm;
    const int64_t *nbr_start;
    const int32_t *nbr_idx;
    const int64_t *red_start;
    const int64_t *red_row;  // tile-grain layout: first row of each entry's source box (else null)
    const void *src;       // sorted q rows (gather) or redundant rows
    const void *table;     // per-instance G(dd) tables, [n_grids][kTableLen] complex
    int32_t nrhs;
    int32_t conj;          // 1: conj(q) in, conj(u) out
    int32_t comp;          // FP32 payload: 1 = each near box's partial sum added into FP64 per target
    void *u;               // caller order
};
constexpr int kTableLen = 148;   // dd = 0..147 inside a 3x3x3-box neighbourhood of 4^3 boxes
p2p_status launch_green_tables(const double *d_h, const double *d_k, int32_t n_grids, bool fp64,
                               void *table, hipStream_t s);
p2p_status launch_helmholtz(const HelmholtzArgs &a, bool redundant, bool fp64, hipStream_t s);

// Multi-RHS Helmholtz on FP32 matrix cores (helmholtz_mfma.hip).
struct HelmholtzMfmaArgs {
    int64_t L;
    int key_bits;
    const int32_t *leaf_start;
    const uint64_t *leaf_key;
    const int32_t *perm;
    const int64_t *nbr_start;
    const int32_t *nbr_idx;
    const int64_t *red_start;
    const int64_t *red_row;    // tile-grain layout: first row of each entry's source box (else null)
    const float2 *src;         // sorted q rows (gather) or redundant rows, [.][nrhs]
    const float2 *blocks;      // multi-RHS: float4 (Re, Im, Re + Im, Re - Im) G at [n_tables][copies][27][64 src]
                               // [64 tgt] (unit spacing); single RHS: float2 (double2 on the FP64 path) at
                               // [n_tables][27][64 src][16][4] (target 16 r + c at [c][r])
    const float2 *zeros;       // 64 zero rows (an absent neighbour's sources, single RHS; double2 on FP64)
    const double *inst_h;      // per instance: h (FP64 single-RHS path with uploaded parameters)
    int64_t n;                 // points
    double2 *parts;            // single RHS: [2][n] partial results in sorted order (tiles split in two)
    int32_t copies;            // copies of each table; workgroup w reads copy (w / 8) % copies
    const int32_t *inst_table; // per instance: table index
    const float *inst_scale;   // per instance: 1/h
    int32_t *counter;          // [8] work-queue counters, one per XCD slice (zeroed by the launcher)
    int32_t nrhs;
    int32_t conj;
    int32_t comp;              // 1: each near box's FP32 partial product summed into FP64 per target
    float2 *u;                 // caller order [n][nrhs]
};
// Per-call parameters of a grid with at most kInlineGrids instances, passed by
// value in the kernel arguments (no upload, no extra launch): n_grids = 0
// means the device arrays are used instead.
constexpr int kInlineGrids = 8;
constexpr int kHelmColBoxes = 16;           // target boxes (columns) per tile of the single-RHS path
struct HelmInline {
    int32_t n_grids;
    int32_t n_tables;
    int32_t tile_first[kInlineGrids + 1];   // first column tile of each instance
    int32_t leaf_first[kInlineGrids + 1];   // first box (leaf) of each instance
    int32_t itab[kInlineGrids];             // G table of each instance
    float iscale[kInlineGrids];             // 1/h of each instance
    double kh[kInlineGrids];                // k h of each table
    double iscale64[kInlineGrids];          // 1/h of each instance in double (FP64 path)
};
// G blocks for the k h values of d_kh, or of inl.kh when inl.n_grids > 0, in the
// multi-RHS or (cols) the single-RHS layout, followed by 64 zero entries; with
// f64 (single-RHS layout only) the entries are double2.
p2p_status launch_green_blocks(const double *d_kh, const HelmInline &inl, int32_t n_tables, int32_t copies,
                               bool cols, bool f64, void *blocks, hipStream_t s);
p2p_status launch_helmholtz_mfma(const HelmholtzMfmaArgs &a, bool redundant, int waves_per_wg,
                                 int wg_per_cu, int rhs_tile, hipStream_t s);
// Single RHS on matrix cores, target boxes as the columns: tiles of up to 16
// consecutive boxes of one instance, (first leaf, count) pairs; returns their
// number (tiles may be null to count).  Uses blocks, inst_table, inst_scale,
// conj and u of the arguments (copies 1, no work queue).
int32_t helmholtz_cols_tiles(const p2p_grid *grids, int32_t n_grids, int32_t *tiles);
p2p_status launch_helmholtz_mfma_cols(const HelmholtzMfmaArgs &a, const int32_t *tiles, const HelmInline &inl,
                                      int32_t n_tiles, bool redundant, bool fp64, hipStream_t s);

// Locality (locality.hip).
p2p_status launch_locality_stats(const int32_t *leaf_start, const int64_t *nbr_start,
                                 const int32_t *nbr_idx, int64_t L, unsigned long long *sums,
                                 hipStream_t s);

}  // namespace p2p

// ------------------------------------------------------------ device side --
namespace p2pd {

// Spread the low 21 bits of v so that bit b moves to bit 3b.
__host__ __device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
// Inverse of spread3: gather bits 0, 3, 6, ... into the low 21 bits.
__host__ __device__ inline uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return static_cast<uint32_t>(v);
}
__host__ __device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This bijection on [0, n) maps workgroup b so that XCD x = b % 8 owns
// one contiguous range of work items, and neighbouring items (which share
// most of their source rows in Morton order) stay in the same L2.
__device__ inline int64_t xcd_contiguous(int64_t b, int64_t n) {
    const int64_t x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// 1/sqrt(x) in double for finite x >= 2^-1022 (every r^2 + eps^2 the FP64
// kernels form: eps >= 2^-511, or eps = 0 with the zero distance selected
// away and distinct points at least 2^-511 apart, as the interface states):
// the hardware estimate y refined by one third-order step of the
// series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2, which leaves
// an error of order e^3, below double rounding.  No special-case tests.
__device__ inline double rsqrt_normal(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

}  // namespace p2pd
