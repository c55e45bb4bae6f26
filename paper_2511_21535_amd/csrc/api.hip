// C ABI entry points of libp2p: argument validation on the host, workspace
// layout, and the launch sequence of every step.  See include/p2p.h.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "p2p_internal.h"

namespace p2p {

namespace {
thread_local std::string g_err;
}  // namespace

void set_error(const std::string &msg) { g_err = msg; }
p2p_status fail(p2p_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

namespace {

hipStream_t as_stream(p2p_stream_t s) { return static_cast<hipStream_t>(s); }

// Workspace protocol shared by every entry point.  Returns true when the call
// only asked for the size (ws == NULL).
bool ws_query(void *ws, size_t *ws_bytes, const Arena &need, p2p_status *st) {
    if (ws == nullptr) {
        *ws_bytes = need.used;
        *st = P2P_OK;
        return true;
    }
    if (*ws_bytes < need.used) {
        *st = fail(P2P_EINVAL, "workspace too small: need " + std::to_string(need.used) +
                                   " bytes, got " + std::to_string(*ws_bytes));
        return true;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) {
        *st = fail(P2P_EINVAL, "workspace must be 256-byte aligned");
        return true;
    }
    return false;
}

// Steps that read counts back, synchronise or copy from host memory cannot be
// recorded into a HIP graph (a recorded host copy would read freed memory at
// replay): they are refused while `s` is capturing, before any work is queued.
p2p_status no_capture(hipStream_t s, const char *what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return fail(P2P_EHIP, "hipStreamIsCapturing failed");
    if (cs != hipStreamCaptureStatusNone)
        return fail(P2P_EUNSUPPORTED, std::string(what) + " reads back, synchronises or copies from host memory: "
                                                          "it cannot be captured into a graph");
    return P2P_OK;
}

int grid_bits_of(const p2p_grid *grids, int32_t n_grids) {
    int mx = 4;
    for (int32_t g = 0; g < n_grids; ++g) mx = grids[g].n_side > mx ? grids[g].n_side : mx;
    int b = 2;
    while ((1 << b) < mx) ++b;
    return b;
}

int bits_for(int64_t v) {  // smallest b with 2^b >= v (v >= 1)
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

p2p_status check_grids(const p2p_grid *grids, int32_t n_grids, int64_t n) {
    if (!grids || n_grids <= 0) return fail(P2P_EINVAL, "grids: need at least one instance");
    int64_t off = 0;
    for (int32_t g = 0; g < n_grids; ++g) {
        const p2p_grid &G = grids[g];
        if (G.n_side < 4 || G.n_side > 1024 || G.n_side % 4 != 0)
            return fail(P2P_EINVAL, "grids[" + std::to_string(g) + "].n_side must be a multiple of 4 in 4..1024");
        if (G.reserved != 0) return fail(P2P_EINVAL, "grids[].reserved must be 0");
        if (!(G.h > 0.0) || !std::isfinite(G.h)) return fail(P2P_EINVAL, "grids[].h must be > 0");
        if (!(G.k >= 0.0) || !std::isfinite(G.k)) return fail(P2P_EINVAL, "grids[].k must be >= 0");
        if (G.point_off != off)
            return fail(P2P_EINVAL, "grids[" + std::to_string(g) + "].point_off must be " + std::to_string(off));
        off += static_cast<int64_t>(G.n_side) * G.n_side * G.n_side;
    }
    if (off != n) return fail(P2P_EINVAL, "grid points (" + std::to_string(off) + ") != tree->n (" + std::to_string(n) + ")");
    return P2P_OK;
}

p2p_status check_tree(const p2p_tree *t) {
    if (!t) return fail(P2P_EINVAL, "tree is NULL");
    if (t->n < 0 || t->n_leaves < 0 || t->n_leaves > t->n) return fail(P2P_EINVAL, "tree: bad sizes (not built?)");
    if (t->n > 0 && (!t->perm || !t->iperm || !t->leaf_start || !t->leaf_key || !t->leaf_level))
        return fail(P2P_EINVAL, "tree: NULL array");
    if (t->kind != P2P_TREE_PARTICLES && t->kind != P2P_TREE_GRIDS) return fail(P2P_EINVAL, "tree: bad kind");
    return P2P_OK;
}

p2p_status check_periodic(const p2p_tree *t, const p2p_nbrs *nb) {
    if (nb->periodic != 0 && nb->periodic != 1) return fail(P2P_EINVAL, "nbrs->periodic must be 0 or 1");
    if (nb->reserved != 0) return fail(P2P_EINVAL, "nbrs->reserved must be 0");
    if (nb->periodic && t->kind != P2P_TREE_PARTICLES)
        return fail(P2P_EINVAL, "periodic near lists are defined for particle trees only");
    return P2P_OK;
}

// remote: lists over another tree's leaves, which may be empty (a plain list
// always holds the leaf itself)
p2p_status check_nbrs(const p2p_tree *t, const p2p_nbrs *nb, bool remote = false) {
    if (!nb) return fail(P2P_EINVAL, "nbrs is NULL");
    P2P_TRY(check_periodic(t, nb));
    if (t->n_leaves > 0 && (!nb->nbr_start || (!remote && !nb->nbr_idx)))
        return fail(P2P_EINVAL, "nbrs: NULL array (not built?)");
    if (nb->count > 0 && (!nb->nbr_idx || (nb->periodic && !nb->nbr_shift)))
        return fail(P2P_EINVAL, "nbrs: NULL nbr_idx or nbr_shift (not built?)");
    if (nb->count < (remote ? 0 : t->n_leaves)) return fail(P2P_EINVAL, "nbrs: count < n_leaves (not built?)");
    return P2P_OK;
}

p2p_status check_remote_trees(const p2p_tree *tree, const p2p_tree *src_tree) {
    P2P_TRY(check_tree(tree));
    if (!src_tree) return fail(P2P_EINVAL, "src_tree is NULL");
    P2P_TRY(check_tree(src_tree));
    if (src_tree == tree) return fail(P2P_EINVAL, "src_tree must be another tree");
    if (tree->kind != P2P_TREE_PARTICLES || src_tree->kind != P2P_TREE_PARTICLES)
        return fail(P2P_EINVAL, "remote interactions need two particle trees");
    return P2P_OK;
}

// Softening length of the gravity sums.  eps == 0 drops pairs at zero
// distance.  A positive eps keeps every pair of distinct points.  FP64 drops
// the target's own pair by position, so any positive eps whose square is a
// normal double (eps >= 2^-511) is exact to rounding.  FP32_MIXED sums the
// target's own d = 0 term m_i / eps into a float partial of at most 32 pair
// terms and subtracts it again afterwards, so the rounding of that partial,
// up to about 32 * 2^-24 m_i / eps, stays in phi_i.  Against a near-field
// potential of a few thousand m_i (a sparse target: tens of neighbours at a
// few hundredths) that stays within 1e-5 relative for eps >= 1e-4; smaller
// positive eps is refused in FP32_MIXED rather than summed inexactly (eps ==
// 0, or FP64, remain available).  The FP32_MIXED adjoint needs eps >= 1e-3:
// its position gradient carries w^5 (d . g) d terms of close pairs, whose
// float rounding measured 2.9e-5 relative at eps = 1e-4 on a 3000-particle
// Plummer mixture (leaf cap 64) and stays within 1e-5 at 1e-3.
constexpr double kMinEpsMixed = 1e-4;
constexpr double kMinEpsMixedAdjoint = 1e-3;
constexpr double kMinEpsFp64 = 0x1p-511;

// adjoint: the gravity adjoint's bounds (eps > 0, and 1e-3 in FP32_MIXED)
p2p_status check_eps(double eps, bool mixed, bool adjoint = false) {
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(P2P_EINVAL, "eps must be finite and >= 0");
    if (adjoint && eps == 0.0) return fail(P2P_EINVAL, "the gravity adjoint needs eps > 0");
    const double lo = mixed ? (adjoint ? kMinEpsMixedAdjoint : kMinEpsMixed) : kMinEpsFp64;
    if (eps > 0.0 && eps < lo)
        return fail(P2P_EINVAL, std::string("eps must be 0 or >= ") +
                                    (mixed ? (adjoint ? "1e-3 with P2P_FP32_MIXED in the adjoint"
                                                      : "1e-4 with P2P_FP32_MIXED")
                                           : "2^-511 (eps^2 a normal double) with P2P_FP64"));
    return P2P_OK;
}

// Precision of the gravity paths: FP64 or FP32_MIXED (P2P_FP32, single
// precision throughout, is provided for the Helmholtz paths only).
p2p_status check_gravity_prec(p2p_precision prec) {
    if (prec == P2P_FP32) return fail(P2P_EUNSUPPORTED, "P2P_FP32 is provided for the Helmholtz paths only");
    if (prec != P2P_FP64 && prec != P2P_FP32_MIXED) return fail(P2P_EINVAL, "bad precision");
    return P2P_OK;
}

// Image codes of periodic lists, null for plain ones.
const int8_t *shifts(const p2p_nbrs *nb) { return nb->periodic ? nb->nbr_shift : nullptr; }

}  // namespace
}  // namespace p2p

using namespace p2p;

extern "C" const char *p2p_last_error(void) { return g_err.c_str(); }
extern "C" const char *p2p_version(void) { return "libp2p 0.1.0 (gfx950)"; }

// ---------------------------------------------------------------- tree ----
extern "C" p2p_status p2p_build_tree(const double *x, const double *y, const double *z,
                                     const p2p_grid *grids, int32_t n_grids, int32_t depth,
                                     int32_t leaf_cap, p2p_tree *tree, void *ws, size_t *ws_bytes,
                                     p2p_stream_t stream) {
    set_error("");
    if (!tree || !ws_bytes) return fail(P2P_EINVAL, "tree and ws_bytes must not be NULL");
    const int64_t n = tree->n;
    if (n < 0) return fail(P2P_EINVAL, "tree->n < 0");
    if (n > INT32_MAX) return fail(P2P_EINVAL, "tree->n exceeds 2^31-1");
    const bool particles = (grids == nullptr);
    int key_bits, sort_bits, leaf_depth = depth;
    if (particles) {
        if (n_grids != 0) return fail(P2P_EINVAL, "n_grids must be 0 for particles");
        if (n > 0 && (!x || !y || !z)) return fail(P2P_EINVAL, "x, y, z must not be NULL");
        if (leaf_cap < 0) return fail(P2P_EINVAL, "leaf_cap < 0");
        if (depth < 0 || depth > 20) return fail(P2P_EINVAL, "depth must be in 0..20");
        key_bits = 20;
        sort_bits = 60;
    } else {
        if (x || y || z) return fail(P2P_EINVAL, "x, y, z must be NULL for grids");
        P2P_TRY(check_grids(grids, n_grids, n));
        key_bits = grid_bits_of(grids, n_grids);
        sort_bits = 3 * key_bits + bits_for(n_grids);
        if (sort_bits > 63) return fail(P2P_EINVAL, "grid key space exceeds 63 bits");
        leaf_depth = key_bits - 2;
    }
    if (tree->cap_leaves < 0) return fail(P2P_EINVAL, "cap_leaves < 0");

    Arena ar(ws);
    uint64_t *keys = ar.take<uint64_t>(n);
    uint64_t *keys_tmp = ar.take<uint64_t>(n);
    int32_t *vals = ar.take<int32_t>(n);
    int32_t *vals_tmp = ar.take<int32_t>(n);
    uint32_t *hist = ar.take<uint32_t>(radix_hist_elems(n));
    uint8_t *pair_common = ar.take<uint8_t>(n);
    int8_t *level = ar.take<int8_t>(n);
    int32_t *flags = ar.take<int32_t>(n);
    int32_t *flag_scan = ar.take<int32_t>(n + 1);
    int32_t *scan_tmp = ar.take<int32_t>(scan_ws_elems(n));
    int32_t *counters = ar.take<int32_t>(2);   // [0] domain flag, [1] max level
    int32_t *d_nside = ar.take<int32_t>(particles ? 1 : n_grids);
    int64_t *d_off = ar.take<int64_t>(particles ? 1 : n_grids);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (n > 0 && (!tree->perm || !tree->iperm || !tree->leaf_start || !tree->leaf_key || !tree->leaf_level))
        return fail(P2P_EINVAL, "tree arrays must not be NULL");
    if (!tree->leaf_start) return fail(P2P_EINVAL, "tree->leaf_start must not be NULL");
    hipStream_t s = as_stream(stream);
    P2P_TRY(no_capture(s, "p2p_build_tree"));

    tree->kind = particles ? P2P_TREE_PARTICLES : P2P_TREE_GRIDS;
    tree->key_bits = key_bits;
    tree->n_grids = particles ? 0 : n_grids;
    if (n == 0) {
        const int32_t zero = 0;
        P2P_HIP(hipMemcpyAsync(tree->leaf_start, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
        P2P_HIP(hipStreamSynchronize(s));
        tree->n_leaves = 0;
        tree->max_level = 0;
        return P2P_OK;
    }
    P2P_HIP(hipMemsetAsync(counters, 0, 2 * sizeof(int32_t), s));
    if (particles) {
        P2P_TRY(launch_particle_keys(x, y, z, n, keys, vals, &counters[0], s));
    } else {
        std::vector<int32_t> ns(n_grids);
        std::vector<int64_t> off(n_grids);
        for (int32_t g = 0; g < n_grids; ++g) {
            ns[g] = grids[g].n_side;
            off[g] = grids[g].point_off;
        }
        P2P_HIP(hipMemcpyAsync(d_nside, ns.data(), n_grids * sizeof(int32_t), hipMemcpyHostToDevice, s));
        P2P_HIP(hipMemcpyAsync(d_off, off.data(), n_grids * sizeof(int64_t), hipMemcpyHostToDevice, s));
        P2P_TRY(launch_grid_keys(d_nside, d_off, n_grids, key_bits, n, keys, vals, s));
    }
    P2P_TRY(radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, n, sort_bits, hist, s));
    P2P_TRY(launch_leaf_levels(keys, n, tree->kind, leaf_depth, particles ? leaf_cap : 0, pair_common,
                               level, flags, s));
    P2P_TRY((exclusive_scan<int32_t, int32_t>(flags, flag_scan, n, scan_tmp, s)));
    int32_t host[2] = {0, 0};
    P2P_HIP(hipMemcpyAsync(&host[0], &flag_scan[n], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipMemcpyAsync(&host[1], &counters[0], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
    const int64_t L = host[0];
    if (host[1] != 0) {
        tree->n_leaves = 0;
        return fail(P2P_EDOMAIN, "a particle coordinate lies outside [0,1) or is NaN");
    }
    if (L > tree->cap_leaves) {
        tree->n_leaves = L;
        return fail(P2P_ECAPACITY, "cap_leaves " + std::to_string(tree->cap_leaves) + " < " + std::to_string(L) + " leaves");
    }
    P2P_TRY(launch_leaf_write(keys, level, flags, flag_scan, n, tree->kind, tree->leaf_start,
                              tree->leaf_key, tree->leaf_level, &counters[1], s));
    P2P_TRY(launch_perm_and_inverse(vals, n, tree->perm, tree->iperm, s));
    int32_t maxl = 0;
    P2P_HIP(hipMemcpyAsync(&maxl, &counters[1], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
    tree->n_leaves = L;
    tree->max_level = maxl;
    return P2P_OK;
}

// ---------------------------------------------------------- near lists ----
namespace p2p {
namespace {

// Near lists of the leaves of `tree` over the leaves of `src` (the same tree for
// plain lists, another particle tree for remote lists).
p2p_status neighbors_common(const p2p_tree *tree, const p2p_tree *src, p2p_nbrs *nbrs, void *ws,
                            size_t *ws_bytes, hipStream_t s) {
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    P2P_TRY(check_tree(tree));
    const bool remote = src != tree;
    if (remote) {
        P2P_TRY(check_tree(src));
        if (tree->kind != P2P_TREE_PARTICLES || src->kind != P2P_TREE_PARTICLES)
            return fail(P2P_EINVAL, "remote lists need two particle trees");
    }
    if (!nbrs) return fail(P2P_EINVAL, "nbrs is NULL");
    if (nbrs->cap < 0) return fail(P2P_EINVAL, "nbrs->cap < 0");
    P2P_TRY(check_periodic(tree, nbrs));
    const bool per = nbrs->periodic != 0;
    const int64_t L = tree->n_leaves, Ls = src->n_leaves;
    // total key bits: 3 per axis, plus the instance index for grids
    const int total_bits = 3 * src->key_bits + (src->kind == P2P_TREE_GRIDS ? bits_for(src->n_grids) : 0);
    Arena ar(ws);
    int32_t *counts = ar.take<int32_t>(L);
    int64_t *start = ar.take<int64_t>(L + 1);
    int64_t *scan_tmp = ar.take<int64_t>(scan_ws_elems(L));
    int32_t *dir = ar.take<int32_t>((size_t(1) << neighbor_dir_bits(total_bits)) + 1);
    int32_t *segs = ar.take<int32_t>(L);
    int64_t *seg_scan = ar.take<int64_t>(L + 1);
    int32_t *slots = ar.take<int32_t>(static_cast<size_t>(L) * kNbrSlotsPerLeaf);
    int8_t *slot_code = ar.take<int8_t>(per ? static_cast<size_t>(L) * kNbrSlotsPerLeaf : 0);
    int32_t *counters = ar.take<int32_t>(2);
    int32_t *heavy = ar.take<int32_t>(L);
    int64_t *totals = ar.take<int64_t>(3);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (!nbrs->nbr_start) return fail(P2P_EINVAL, "nbrs->nbr_start must not be NULL");
    P2P_TRY(no_capture(s, "building near lists"));
    const int inst_shift = 3 * src->key_bits;
    const NbrTargets tg{tree->leaf_key, tree->leaf_level, L};
    const NbrTargets *tgp = remote ? &tg : nullptr;
    P2P_TRY(launch_key_directory(src->leaf_key, Ls, total_bits, dir, counters, s));
    P2P_TRY(launch_neighbors_count(src->leaf_key, src->leaf_level, Ls, src->key_bits, inst_shift, dir,
                                   total_bits, src->leaf_start, counts, segs, slots,
                                   per ? slot_code : nullptr, counters, heavy, s, tgp));
    P2P_TRY((exclusive_scan<int32_t, int64_t>(counts, start, L, scan_tmp, s)));
    P2P_TRY((exclusive_scan<int32_t, int64_t>(segs, seg_scan, L, scan_tmp, s)));
    P2P_TRY(launch_nbr_totals(start, seg_scan, counters, L, totals, s));
    int64_t host[3] = {0, 0, 0};
    P2P_HIP(hipMemcpyAsync(host, totals, sizeof(host), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
    const int64_t E = host[0];
    nbrs->red_entries = host[1];
    if (E > nbrs->cap) {
        nbrs->count = E;
        return fail(P2P_ECAPACITY, "nbrs->cap " + std::to_string(nbrs->cap) + " < " + std::to_string(E) + " entries");
    }
    if (E > 0 && !nbrs->nbr_idx) return fail(P2P_EINVAL, "nbrs->nbr_idx must not be NULL");
    if (E > 0 && per && !nbrs->nbr_shift) return fail(P2P_EINVAL, "nbrs->nbr_shift must not be NULL for periodic lists");
    P2P_HIP(hipMemcpyAsync(nbrs->nbr_start, start, (L + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    P2P_TRY(launch_neighbors_fill(src->leaf_key, src->leaf_level, Ls, src->key_bits, inst_shift, dir,
                                  total_bits, counts, slots, per ? slot_code : nullptr, counters, heavy, host[2] > 0,
                                  nbrs->nbr_start, nbrs->nbr_idx, per ? nbrs->nbr_shift : nullptr, s, tgp));
    P2P_HIP(hipStreamSynchronize(s));
    nbrs->count = E;
    return P2P_OK;
}

}  // namespace
}  // namespace p2p

extern "C" p2p_status p2p_build_neighbors(const p2p_tree *tree, p2p_nbrs *nbrs, void *ws,
                                          size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    return neighbors_common(tree, tree, nbrs, ws, ws_bytes, as_stream(stream));
}

extern "C" p2p_status p2p_build_neighbors_remote(const p2p_tree *tree, const p2p_tree *src_tree,
                                                 p2p_nbrs *nbrs, void *ws, size_t *ws_bytes,
                                                 p2p_stream_t stream) {
    set_error("");
    if (!src_tree) return fail(P2P_EINVAL, "src_tree is NULL");
    if (src_tree == tree) return fail(P2P_EINVAL, "src_tree must be another tree (plain lists: p2p_build_neighbors)");
    return neighbors_common(tree, src_tree, nbrs, ws, ws_bytes, as_stream(stream));
}

// --------------------------------------------------------- restructure ----
namespace p2p {
namespace {

// Segments of the targets of `tree` filled from the points of `srct` (the same
// tree, or the source tree of remote lists).
// Tile grain on a grid tree: halo sizes per tile, their scan, the total read
// back (the capacity check needs it), then the halo lists with the row of
// every near-list entry, and the copy of the halo boxes' rows from caller
// order.
p2p_status restructure_tiles(const p2p_tree *tree, const p2p_nbrs *nbrs, const void *const src[4], int32_t nrhs,
                             p2p_precision prec, p2p_redundant *out, void *ws, size_t *ws_bytes, hipStream_t s) {
    const int grain = out->grain;
    if (grain != 2 && grain != 4) return fail(P2P_EINVAL, "out->grain must be 0, 1 (box grain), 2 or 4 (tiles)");
    const bool mixed = prec != P2P_FP64;
    const int64_t L = tree->n_leaves, E = nbrs->count;
    const int64_t row_bytes = static_cast<int64_t>(nrhs) * (mixed ? 8 : 16);
    Arena ar(ws);
    int64_t *cnt = ar.take<int64_t>(L);
    int64_t *hs = ar.take<int64_t>(L + 1);
    int64_t *scan_tmp = ar.take<int64_t>(scan_ws_elems(L));
    int32_t *halo = ar.take<int32_t>(E);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (!src || (tree->n > 0 && !src[0])) return fail(P2P_EINVAL, "src[0] (q) must not be NULL");
    if (!out->red_start || (E > 0 && !out->red_row)) return fail(P2P_EINVAL, "out->red_start/red_row must not be NULL");
    if (out->cap < 0) return fail(P2P_EINVAL, "out->cap < 0");
    P2P_TRY(no_capture(s, "a tile-grain restructure"));
    P2P_TRY(launch_tile_halo(tree->leaf_key, nbrs->nbr_start, nbrs->nbr_idx, L, tree->key_bits, grain, cnt,
                             nullptr, nullptr, nullptr, nullptr, s));
    P2P_TRY((exclusive_scan<int64_t, int64_t>(cnt, hs, L, scan_tmp, s)));
    int64_t H = 0;
    if (L > 0) P2P_HIP(hipMemcpyAsync(&H, hs + L, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
    const int64_t S = 64 * H;
    if (S > out->cap) {
        out->count = S;
        return fail(P2P_ECAPACITY, "out->cap " + std::to_string(out->cap) + " < " + std::to_string(S) + " entries");
    }
    if (S > 0 && !out->planes[0]) return fail(P2P_EINVAL, "out->planes must not be NULL");
    P2P_TRY(launch_tile_halo(tree->leaf_key, nbrs->nbr_start, nbrs->nbr_idx, L, tree->key_bits, grain, nullptr,
                             hs, halo, out->red_row, out->red_start, s));
    P2P_TRY(launch_tile_copy(src[0], row_bytes, tree->leaf_start, tree->perm, halo, H, out->planes[0],
                             S * row_bytes > kStreamingLayoutBytes, s));
    out->count = S;
    out->nrhs = nrhs;
    out->kind = P2P_KIND_HELMHOLTZ;
    out->prec = prec;
    return P2P_OK;
}

p2p_status restructure_common(const p2p_tree *tree, const p2p_tree *srct, const p2p_nbrs *nbrs,
                              const void *const src[4], int32_t nrhs, p2p_precision prec, p2p_redundant *out,
                              void *ws, size_t *ws_bytes, hipStream_t s) {
    const bool remote = srct != tree;
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    if (remote)
        P2P_TRY(check_remote_trees(tree, srct));
    else
        P2P_TRY(check_tree(tree));
    P2P_TRY(check_nbrs(tree, nbrs, remote));
    if (!out) return fail(P2P_EINVAL, "out is NULL");
    const bool grav = tree->kind == P2P_TREE_PARTICLES;
    if (grav) P2P_TRY(check_gravity_prec(prec));
    else if (prec != P2P_FP64 && prec != P2P_FP32_MIXED && prec != P2P_FP32) return fail(P2P_EINVAL, "bad precision");
    if (!grav && nrhs < 1) return fail(P2P_EINVAL, "nrhs must be >= 1");
    if (grav) nrhs = 1;
    if (out->grain != 0 && out->grain != 1) {
        if (grav || remote) return fail(P2P_EINVAL, "out->grain > 1 (tiles) is defined on grid trees only");
        return restructure_tiles(tree, nbrs, src, nrhs, prec, out, ws, ws_bytes, s);
    }
    // single-precision payload: leaf-relative float rows (gravity), complex64 (Helmholtz)
    const bool mixed = prec != P2P_FP64;
    // n: the source rows; L: the target leaves
    const int64_t n = srct->n, L = tree->n_leaves;
    const size_t csize = mixed ? sizeof(float2) : sizeof(double2);
    Arena ar(ws);
    int32_t *seg_len = ar.take<int32_t>(L);
    int64_t *scan_tmp = ar.take<int64_t>(scan_ws_elems(L));
    int64_t *count_start = ar.take<int64_t>(nbrs->red_entries < 0 ? L + 1 : 0);
    int32_t *count_self = ar.take<int32_t>(nbrs->red_entries < 0 ? L : 0);
    Row4d *s4 = nullptr;
    void *sq = nullptr;
    if (grav) {
        if (!remote) s4 = ar.take<Row4d>(n);
    } else {
        sq = ar.take<char>(static_cast<size_t>(n) * nrhs * csize);
    }
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (!src) return fail(P2P_EINVAL, "src is NULL");
    if (n > 0 && (grav ? (!src[0] || !src[1] || !src[2] || !src[3]) : !src[0]))
        return fail(P2P_EINVAL, "src arrays must not be NULL");
    if (!out->red_start || (L > 0 && !out->red_self)) return fail(P2P_EINVAL, "out->red_start/red_self must not be NULL");
    if (out->cap < 0) return fail(P2P_EINVAL, "out->cap < 0");
    // S: carried by the near lists, else counted here and read back
    int64_t S = nbrs->red_entries;
    if (S < 0) {
        P2P_TRY(no_capture(s, "a restructure over near lists without their size"));
        P2P_TRY(launch_seg_lengths(srct->leaf_start, nbrs->nbr_start, nbrs->nbr_idx, shifts(nbrs), L, seg_len,
                                   count_self, !remote, s));
        P2P_TRY((exclusive_scan<int32_t, int64_t>(seg_len, count_start, L, scan_tmp, s)));
        S = 0;
        if (L > 0) P2P_HIP(hipMemcpyAsync(&S, &count_start[L], sizeof(int64_t), hipMemcpyDeviceToHost, s));
        P2P_HIP(hipStreamSynchronize(s));
    }
    if (S > out->cap) {
        out->count = S;
        return fail(P2P_ECAPACITY, "out->cap " + std::to_string(out->cap) + " < " + std::to_string(S) + " entries");
    }
    if (S > 0 && !out->planes[0])
        return fail(P2P_EINVAL, "out->planes must not be NULL");
    // rows into sorted order first: the longest of the short launches, so the
    // segment offsets below are already queued when it ends.  Remote sources
    // are not sorted: the copy reads them through the source tree's perm (a
    // thin layer of the other domain is used)
    const PermRows pr{static_cast<const double *>(src[0]), static_cast<const double *>(src[1]),
                      static_cast<const double *>(src[2]), static_cast<const double *>(src[3]), srct->perm};
    if (grav) {
        if (!remote)
            P2P_TRY(launch_scatter4(static_cast<const double *>(src[0]), static_cast<const double *>(src[1]),
                                    static_cast<const double *>(src[2]), static_cast<const double *>(src[3]),
                                    srct->iperm, n, s4, s));
    } else if (mixed)
        P2P_TRY(launch_permute_rows<float2>(static_cast<const float2 *>(src[0]), tree->perm, n, nrhs,
                                            static_cast<float2 *>(sq), s));
    else
        P2P_TRY(launch_permute_rows<double2>(static_cast<const double2 *>(src[0]), tree->perm, n, nrhs,
                                             static_cast<double2 *>(sq), s));
    // grid boxes all hold 64 points: the copy writes the segment offsets itself
    BoxSegments boxes{};
    if (tree->kind == P2P_TREE_GRIDS) {
        boxes.red_start = out->red_start;
        boxes.red_self = out->red_self;
        boxes.box_rows = 64;
        boxes.entries = nbrs->count;
        if (L == 0) P2P_TRY((exclusive_scan<int32_t, int64_t>(seg_len, out->red_start, 0, scan_tmp, s)));
    } else {
        P2P_TRY(launch_seg_lengths(srct->leaf_start, nbrs->nbr_start, nbrs->nbr_idx, shifts(nbrs), L, seg_len,
                                   out->red_self, !remote, s));
        P2P_TRY((exclusive_scan<int32_t, int64_t>(seg_len, out->red_start, L, scan_tmp, s)));
    }
    const int64_t entry_bytes = grav ? (mixed ? 16 : 32) : static_cast<int64_t>(nrhs) * static_cast<int64_t>(csize);
    const bool streaming = S * entry_bytes > kStreamingLayoutBytes;
    if (grav)
        P2P_TRY(launch_copy_segments_gravity(s4, tree->leaf_key, tree->leaf_level, srct->leaf_start,
                                             nbrs->nbr_start, nbrs->nbr_idx, shifts(nbrs), out->red_start, L,
                                             mixed ? nullptr : static_cast<Row4d *>(out->planes[0]),
                                             mixed ? static_cast<float4 *>(out->planes[0]) : nullptr,
                                             streaming, s, remote ? &pr : nullptr));
    else if (mixed)
        P2P_TRY(launch_copy_segments<float2>(static_cast<const float2 *>(sq), nrhs, tree->leaf_start,
                                             nbrs->nbr_start, nbrs->nbr_idx, out->red_start, L,
                                             static_cast<float2 *>(out->planes[0]), streaming, s, boxes));
    else
        P2P_TRY(launch_copy_segments<double2>(static_cast<const double2 *>(sq), nrhs, tree->leaf_start,
                                              nbrs->nbr_start, nbrs->nbr_idx, out->red_start, L,
                                              static_cast<double2 *>(out->planes[0]), streaming, s, boxes));
    out->count = S;
    out->nrhs = nrhs;
    out->kind = grav ? P2P_KIND_GRAVITY : P2P_KIND_HELMHOLTZ;
    out->prec = prec;
    return P2P_OK;
}

}  // namespace
}  // namespace p2p

extern "C" p2p_status p2p_restructure_redundant(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                                const void *const src[4], int32_t nrhs,
                                                p2p_precision prec, p2p_redundant *out, void *ws,
                                                size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    return restructure_common(tree, tree, nbrs, src, nrhs, prec, out, ws, ws_bytes, as_stream(stream));
}

extern "C" p2p_status p2p_restructure_remote(const p2p_tree *tree, const p2p_tree *src_tree,
                                             const p2p_nbrs *nbrs, const double *const src[4],
                                             p2p_precision prec, p2p_redundant *out, void *ws,
                                             size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!src_tree) return fail(P2P_EINVAL, "src_tree is NULL");
    const void *const s4[4] = {src ? src[0] : nullptr, src ? src[1] : nullptr, src ? src[2] : nullptr,
                               src ? src[3] : nullptr};
    return restructure_common(tree, src_tree, nbrs, src ? s4 : nullptr, 1, prec, out, ws, ws_bytes,
                              as_stream(stream));
}

// ------------------------------------------------- per-interaction layout ---
extern "C" p2p_status p2p_restructure_interactions(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                                   const double *const src[4], p2p_precision prec,
                                                   p2p_interactions *out, void *ws, size_t *ws_bytes,
                                                   p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    P2P_TRY(check_tree(tree));
    if (tree->kind != P2P_TREE_PARTICLES) return fail(P2P_EINVAL, "the per-interaction layout needs a particle tree");
    P2P_TRY(check_nbrs(tree, nbrs));
    if (!out) return fail(P2P_EINVAL, "out is NULL");
    P2P_TRY(check_gravity_prec(prec));
    const bool mixed = prec == P2P_FP32_MIXED;
    const int64_t n = tree->n, L = tree->n_leaves, E = nbrs->count;
    const bool known = nbrs->red_entries >= 0;
    Arena ar(ws);
    Row4d *s4 = ar.take<Row4d>(n);
    int32_t *rec_len = ar.take<int32_t>(E);
    int32_t *tgt_len = ar.take<int32_t>(known ? 0 : E);
    int64_t *tgt_scan = ar.take<int64_t>(known ? 0 : E + 1);
    int64_t *scan_tmp = ar.take<int64_t>(scan_ws_elems(E));
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (!src || (n > 0 && (!src[0] || !src[1] || !src[2] || !src[3])))
        return fail(P2P_EINVAL, "src arrays must not be NULL");
    if (!out->rec_start) return fail(P2P_EINVAL, "out->rec_start must not be NULL");
    if (out->cap < 0) return fail(P2P_EINVAL, "out->cap < 0");
    hipStream_t s = as_stream(stream);
    if (!known) P2P_TRY(no_capture(s, "an interaction restructure over near lists without their size"));
    P2P_TRY(launch_scatter4(src[0], src[1], src[2], src[3], tree->iperm, n, s4, s));
    // rows: E headers plus, per record, its targets and sources; with the
    // symmetric lists of p2p_build_neighbors both sums are S
    int64_t rows = 0, trows = 0;
    if (known) {
        rows = E + 2 * nbrs->red_entries;
        trows = nbrs->red_entries;
    } else {
        P2P_TRY(launch_record_lengths(tree->leaf_start, nbrs->nbr_start, nbrs->nbr_idx, L, rec_len, tgt_len, s));
        P2P_TRY((exclusive_scan<int32_t, int64_t>(rec_len, out->rec_start, E, scan_tmp, s)));
        P2P_TRY((exclusive_scan<int32_t, int64_t>(tgt_len, tgt_scan, E, scan_tmp, s)));
        if (E > 0) {
            P2P_HIP(hipMemcpyAsync(&rows, &out->rec_start[E], sizeof(int64_t), hipMemcpyDeviceToHost, s));
            P2P_HIP(hipMemcpyAsync(&trows, &tgt_scan[E], sizeof(int64_t), hipMemcpyDeviceToHost, s));
        }
        P2P_HIP(hipStreamSynchronize(s));
    }
    if (rows > out->cap) {
        out->count = rows;
        return fail(P2P_ECAPACITY, "out->cap " + std::to_string(out->cap) + " < " + std::to_string(rows) + " rows");
    }
    if (rows > 0 && !out->planes[0]) return fail(P2P_EINVAL, "out->planes[0] must not be NULL");
    if (known) {
        P2P_TRY(launch_record_lengths(tree->leaf_start, nbrs->nbr_start, nbrs->nbr_idx, L, rec_len, nullptr, s));
        P2P_TRY((exclusive_scan<int32_t, int64_t>(rec_len, out->rec_start, E, scan_tmp, s)));
    }
    const bool streaming = rows * (mixed ? 16 : 32) > kStreamingLayoutBytes;
    P2P_TRY(launch_copy_records(s4, tree->leaf_key, tree->leaf_level, tree->leaf_start, nbrs->nbr_start,
                                nbrs->nbr_idx, shifts(nbrs), out->rec_start, L,
                                mixed ? nullptr : static_cast<Row4d *>(out->planes[0]),
                                mixed ? static_cast<float4 *>(out->planes[0]) : nullptr, streaming, s));
    out->count = rows;
    out->target_rows = trows;
    out->prec = prec;
    return P2P_OK;
}

extern "C" p2p_status p2p_eval_gravity_interactions(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                                    const p2p_interactions *inter, double eps,
                                                    double *phi, double *ax, double *ay, double *az,
                                                    void *ws, size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    P2P_TRY(check_tree(tree));
    if (tree->kind != P2P_TREE_PARTICLES) return fail(P2P_EINVAL, "gravity needs a particle tree");
    P2P_TRY(check_nbrs(tree, nbrs));
    if (!inter) return fail(P2P_EINVAL, "inter is NULL");
    if (inter->prec != P2P_FP64 && inter->prec != P2P_FP32_MIXED) return fail(P2P_EINVAL, "inter was not built");
    if (inter->target_rows < 0) return fail(P2P_EINVAL, "inter->target_rows < 0");
    const bool mixed = inter->prec == P2P_FP32_MIXED;
    P2P_TRY(check_eps(eps, mixed));
    const int64_t n = tree->n, L = tree->n_leaves, E = nbrs->count;
    Arena ar(ws);
    int32_t *tgt_len = ar.take<int32_t>(E);
    int64_t *res_start = ar.take<int64_t>(E + 1);
    int64_t *scan_tmp = ar.take<int64_t>(scan_ws_elems(E));
    Row4d *res = ar.take<Row4d>(inter->target_rows);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (n > 0 && (!phi || !ax || !ay || !az)) return fail(P2P_EINVAL, "outputs must not be NULL");
    if (!inter->rec_start || (inter->count > 0 && !inter->planes[0]))
        return fail(P2P_EINVAL, "inter arrays must not be NULL");
    hipStream_t s = as_stream(stream);
    P2P_TRY(launch_record_lengths(tree->leaf_start, nbrs->nbr_start, nbrs->nbr_idx, L, nullptr, tgt_len, s));
    P2P_TRY((exclusive_scan<int32_t, int64_t>(tgt_len, res_start, E, scan_tmp, s)));
    P2P_TRY(launch_eval_records(inter->rec_start, mixed ? nullptr : static_cast<const Row4d *>(inter->planes[0]),
                                mixed ? static_cast<const float4 *>(inter->planes[0]) : nullptr, shifts(nbrs), E,
                                res_start, eps * eps, eps == 0.0, res, s));
    P2P_TRY(launch_reduce_records(tree->leaf_start, nbrs->nbr_start, res_start, tree->perm, L, res, phi, ax,
                                  ay, az, s));
    return P2P_OK;
}

// ------------------------------------------------------------- gravity ----
namespace p2p {

p2p_status gravity_check_args(const p2p_tree *tree, const p2p_nbrs *nbrs, p2p_layout layout,
                              p2p_precision prec, double eps) {
    P2P_TRY(check_tree(tree));
    if (tree->kind != P2P_TREE_PARTICLES) return fail(P2P_EINVAL, "gravity needs a particle tree");
    P2P_TRY(check_nbrs(tree, nbrs));
    if (layout != P2P_GATHER && layout != P2P_REDUNDANT) return fail(P2P_EINVAL, "bad layout");
    P2P_TRY(check_gravity_prec(prec));
    return check_eps(eps, prec == P2P_FP32_MIXED);
}

p2p_status gravity_run(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                       p2p_layout layout, p2p_precision prec, double eps, const double *x,
                       const double *y, const double *z, const double *m, double *phi, double *ax,
                       double *ay, double *az, Row4d *s4, hipStream_t s) {
    const bool mixed = prec == P2P_FP32_MIXED, redundant = layout == P2P_REDUNDANT;
    const int64_t n = tree->n;
    if (n > 0 && (!phi || !ax || !ay || !az)) return fail(P2P_EINVAL, "outputs must not be NULL");
    if (redundant) {
        if (!red) return fail(P2P_EINVAL, "REDUNDANT layout needs red");
        if (red->kind != P2P_KIND_GRAVITY) return fail(P2P_EINVAL, "red was not built for gravity");
        if (red->prec != prec) return fail(P2P_EINVAL, "red was built with another precision");
        if (!red->red_start || !red->red_self || (red->count > 0 && !red->planes[0]))
            return fail(P2P_EINVAL, "red arrays must not be NULL");
    } else if (n > 0 && (!x || !y || !z || !m)) {
        return fail(P2P_EINVAL, "GATHER layout needs x, y, z, m");
    }
    GravityArgs a{};
    a.L = tree->n_leaves;
    a.leaf_start = tree->leaf_start;
    a.src_leaf_start = tree->leaf_start;
    a.perm = tree->perm;
    a.leaf_key = tree->leaf_key;
    a.leaf_level = tree->leaf_level;
    a.nbr_start = nbrs->nbr_start;
    a.nbr_idx = nbrs->nbr_idx;
    a.nbr_shift = shifts(nbrs);
    a.eps2 = eps * eps;
    a.phi = phi;
    a.ax = ax;
    a.ay = ay;
    a.az = az;
    if (redundant) {
        a.red_start = red->red_start;
        a.red_self = red->red_self;
        if (mixed)
            a.red4 = static_cast<const float4 *>(red->planes[0]);
        else
            a.s4 = static_cast<const Row4d *>(red->planes[0]);
    } else {
        P2P_TRY(launch_scatter4(x, y, z, m, tree->iperm, n, s4, s));
        a.s4 = s4;
    }
    return launch_gravity(a, redundant, mixed, eps == 0.0, s);
}

}  // namespace p2p

extern "C" p2p_status p2p_eval_gravity(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                       const p2p_redundant *red, p2p_layout layout,
                                       p2p_precision prec, double eps, const double *x,
                                       const double *y, const double *z, const double *m,
                                       double *phi, double *ax, double *ay, double *az, void *ws,
                                       size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    P2P_TRY(gravity_check_args(tree, nbrs, layout, prec, eps));
    Arena ar(ws);
    Row4d *s4 = layout == P2P_REDUNDANT ? nullptr : ar.take<Row4d>(tree->n);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    return gravity_run(tree, nbrs, red, layout, prec, eps, x, y, z, m, phi, ax, ay, az, s4, as_stream(stream));
}

extern "C" p2p_status p2p_eval_gravity_remote(const p2p_tree *tree, const p2p_tree *src_tree,
                                              const p2p_nbrs *nbrs, const p2p_redundant *red,
                                              p2p_layout layout, p2p_precision prec, double eps,
                                              const double *x, const double *y, const double *z,
                                              const double *sx, const double *sy, const double *sz,
                                              const double *sm, double *phi, double *ax, double *ay,
                                              double *az, void *ws, size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    P2P_TRY(check_remote_trees(tree, src_tree));
    P2P_TRY(check_nbrs(tree, nbrs, true));
    if (layout != P2P_GATHER && layout != P2P_REDUNDANT) return fail(P2P_EINVAL, "bad layout");
    P2P_TRY(check_gravity_prec(prec));
    const bool mixed = prec == P2P_FP32_MIXED, redundant = layout == P2P_REDUNDANT;
    P2P_TRY(check_eps(eps, mixed));
    const int64_t n = tree->n, ns = src_tree->n;
    Arena ar(ws);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (n > 0 && (!phi || !ax || !ay || !az)) return fail(P2P_EINVAL, "outputs must not be NULL");
    if (n > 0 && (!x || !y || !z)) return fail(P2P_EINVAL, "x, y, z (targets) must not be NULL");
    if (redundant) {
        if (!red) return fail(P2P_EINVAL, "REDUNDANT layout needs red");
        if (red->kind != P2P_KIND_GRAVITY) return fail(P2P_EINVAL, "red was not built for gravity");
        if (red->prec != prec) return fail(P2P_EINVAL, "red was built with another precision");
        if (!red->red_start || (red->count > 0 && !red->planes[0]))
            return fail(P2P_EINVAL, "red arrays must not be NULL");
    } else if (ns > 0 && (!sx || !sy || !sz || !sm)) {
        return fail(P2P_EINVAL, "GATHER layout needs sx, sy, sz, sm");
    }
    hipStream_t s = as_stream(stream);
    GravityArgs a{};
    a.L = tree->n_leaves;
    a.leaf_start = tree->leaf_start;
    a.src_leaf_start = src_tree->leaf_start;
    a.perm = tree->perm;
    a.leaf_key = tree->leaf_key;
    a.leaf_level = tree->leaf_level;
    a.nbr_start = nbrs->nbr_start;
    a.nbr_idx = nbrs->nbr_idx;
    a.nbr_shift = shifts(nbrs);
    a.eps2 = eps * eps;
    a.phi = phi;
    a.ax = ax;
    a.ay = ay;
    a.az = az;
    a.tx = x;
    a.ty = y;
    a.tz = z;
    if (redundant) {
        a.red_start = red->red_start;
        if (mixed)
            a.red4 = static_cast<const float4 *>(red->planes[0]);
        else
            a.s4 = static_cast<const Row4d *>(red->planes[0]);
    } else {
        a.sx = sx;
        a.sy = sy;
        a.sz = sz;
        a.sm = sm;
        a.src_perm = src_tree->perm;
    }
    return launch_gravity_remote(a, redundant, mixed, eps == 0.0, s);
}

// ----------------------------------------------------------- Helmholtz ----
namespace {

// Everything a Helmholtz evaluation derives from its arguments on the host:
// the path (matrix cores multi-RHS or single RHS, or the vector kernel), the
// launch shape, the distinct k h values (one G table or set of G blocks each),
// and the layout of the set-up buffer.  The set-up buffer (the plan) holds the
// instances' parameters and the G tables or blocks; it
// is filled by helm_fill, either on every call (p2p_eval_helmholtz, in the
// workspace) or once (p2p_helmholtz_prepare, in a caller buffer).
struct HelmSetup {
    p2p_precision prec;
    int32_t nrhs;
    bool fp64, mfma, cols, blk, inline_params;
    int waves_per_wg = 4, wg_per_cu = 2, rhs_tile = 32, copies = 1;
    int32_t n_grids = 0, n_tables = 0, n_tiles = 0;
    std::vector<double> khs;
    std::vector<int32_t> itab;
    std::vector<float> iscale;
    size_t o_k = 0, o_kh = 0, o_itab = 0, o_isc = 0, o_tiles = 0, param_bytes = 0;
    HelmInline inl{};
};

// Device arrays of the set-up inside an arena (null pointers when sizing).
struct HelmSetupBufs {
    char *params = nullptr;
    char *table = nullptr;
    float2 *blocks = nullptr;
};

p2p_status helm_setup(const p2p_tree *tree, const p2p_nbrs *nbrs, p2p_precision prec, const p2p_grid *grids,
                      int32_t n_grids, int32_t nrhs, const int32_t *tile, HelmSetup *h) {
    P2P_TRY(check_tree(tree));
    if (tree->kind != P2P_TREE_GRIDS) return fail(P2P_EINVAL, "Helmholtz needs a grid tree");
    P2P_TRY(check_nbrs(tree, nbrs));
    if (prec != P2P_FP64 && prec != P2P_FP32_MIXED && prec != P2P_FP32) return fail(P2P_EINVAL, "bad precision");
    if (nrhs < 1) return fail(P2P_EINVAL, "nrhs must be >= 1");
    if (n_grids != tree->n_grids) return fail(P2P_EINVAL, "n_grids differs from the tree's");
    P2P_TRY(check_grids(grids, n_grids, tree->n));
    h->prec = prec;
    h->nrhs = nrhs;
    h->n_grids = n_grids;
    h->fp64 = prec == P2P_FP64;
    // the matrix-core product addresses a box's 64 source rows with 32-bit byte
    // offsets (buffer loads), so nrhs above 2^20 takes the vector kernel
    h->mfma = !h->fp64 && nrhs % 32 == 0 && nrhs <= (1 << 20);
    // one RHS: matrix cores (FP32, or FP64 on the FP64 matrix instructions) with the target boxes as columns
    h->cols = nrhs == 1;
    h->rhs_tile = (nrhs % 64 == 0) ? 64 : 32;
    if (tile) {
        if (!h->mfma) return fail(P2P_EINVAL, "tile applies to the matrix-core path (FP32_MIXED, nrhs % 32 == 0)");
        h->waves_per_wg = tile[0];
        h->wg_per_cu = tile[1];
        h->rhs_tile = tile[2];
        h->copies = tile[3];
        if (h->copies != 1 && h->copies != 2 && h->copies != 4 && h->copies != 8)
            return fail(P2P_EINVAL, "tile[3] (copies of the G blocks) must be 1, 2, 4 or 8");
        if (h->waves_per_wg != 1 && h->waves_per_wg != 2 && h->waves_per_wg != 4)
            return fail(P2P_EINVAL, "tile[0] (waves per workgroup) must be 1, 2 or 4");
        if (h->wg_per_cu < 1 || h->wg_per_cu > 16) return fail(P2P_EINVAL, "tile[1] (workgroups per CU) must be in 1..16");
        if ((h->rhs_tile != 32 && h->rhs_tile != 64) || nrhs % h->rhs_tile != 0)
            return fail(P2P_EINVAL, "tile[2] (RHS tile) must be 32 or 64 and divide nrhs");
    }
    // distinct k h values share one set of unit-spacing G blocks (relative tolerance 1e-12)
    h->itab.resize(n_grids);
    h->iscale.resize(n_grids);
    for (int32_t g = 0; g < n_grids; ++g) {
        const double kh = grids[g].k * grids[g].h;
        int32_t t = -1;
        for (size_t j = 0; j < h->khs.size(); ++j)
            if (std::fabs(h->khs[j] - kh) <= 1e-12 * std::fmax(std::fabs(kh), 1e-300) || h->khs[j] == kh) {
                t = static_cast<int32_t>(j);
                break;
            }
        if (t < 0) {
            t = static_cast<int32_t>(h->khs.size());
            h->khs.push_back(kh);
        }
        h->itab[g] = t;
        h->iscale[g] = static_cast<float>(1.0 / grids[g].h);
    }
    h->n_tables = static_cast<int32_t>(h->khs.size());
    h->blk = h->mfma || h->cols;
    h->n_tiles = h->cols ? helmholtz_cols_tiles(grids, n_grids, nullptr) : 0;
    if (h->cols) {
        // every box of a grid instance is a leaf, instances in order
        int64_t boxes = 0;
        for (int32_t g = 0; g < n_grids; ++g)
            boxes += static_cast<int64_t>(grids[g].n_side / 4) * (grids[g].n_side / 4) * (grids[g].n_side / 4);
        if (boxes != tree->n_leaves) return fail(P2P_EINVAL, "tree leaves do not match the grids' boxes");
    }
    // the host parameters (h and k per instance, k h per table, the table and
    // 1/h of each instance, the column tiles) travel in one copy: each small
    // copy costs a blit launch, a sizeable part of a call on a small grid
    h->o_k = 8 * static_cast<size_t>(n_grids);
    h->o_kh = h->o_k + 8 * static_cast<size_t>(n_grids);
    h->o_itab = h->o_kh + 8 * static_cast<size_t>(h->n_tables);
    h->o_isc = h->o_itab + 4 * static_cast<size_t>(n_grids);
    h->o_tiles = h->o_isc + 4 * static_cast<size_t>(n_grids);
    h->param_bytes = h->o_tiles + 8 * static_cast<size_t>(h->n_tiles);
    // a single-RHS call on a grid of few instances takes its parameters in the
    // kernel arguments; every other call uploads them
    h->inline_params = h->cols && n_grids <= kInlineGrids && h->n_tables <= kInlineGrids;
    if (h->inline_params) {
        HelmInline &inl = h->inl;
        inl.n_grids = n_grids;
        inl.n_tables = h->n_tables;
        int32_t tf = 0, lf = 0;
        for (int32_t g = 0; g < n_grids; ++g) {
            const int32_t nb = (grids[g].n_side / 4) * (grids[g].n_side / 4) * (grids[g].n_side / 4);
            inl.tile_first[g] = tf;
            inl.leaf_first[g] = lf;
            inl.itab[g] = h->itab[g];
            inl.iscale[g] = h->iscale[g];
            inl.iscale64[g] = 1.0 / grids[g].h;
            tf += (nb + kHelmColBoxes - 1) / kHelmColBoxes;
            lf += nb;
        }
        inl.tile_first[n_grids] = tf;
        inl.leaf_first[n_grids] = lf;
        for (int32_t t = 0; t < h->n_tables; ++t) inl.kh[t] = h->khs[t];
    }
    return P2P_OK;
}

HelmSetupBufs helm_take(Arena &ar, const HelmSetup &h) {
    const size_t csize = h.fp64 ? sizeof(double2) : sizeof(float2);
    HelmSetupBufs b;
    b.params = ar.take<char>(h.param_bytes);
    if (!h.blk) b.table = ar.take<char>(static_cast<size_t>(h.n_grids) * kTableLen * csize);
    // the G blocks: multi-RHS float4 entries; single RHS float2 (FP64: double2) entries and 64 zero
    // entries after them
    if (h.blk)
        b.blocks = ar.take<float2>(h.cols ? (static_cast<size_t>(h.n_tables) * 27 * 4096 + 64) * (h.fp64 ? 2 : 1)
                                          : static_cast<size_t>(h.n_tables) * h.copies * 27 * 4096 * 2);
    return b;
}

// Fill the set-up buffer: parameters uploaded (unless they travel inline),
// the G tables (vector path) or blocks (matrix cores).
p2p_status helm_fill(const HelmSetup &h, const HelmSetupBufs &b, const p2p_tree *tree, const p2p_nbrs *nbrs,
                     const p2p_grid *grids, hipStream_t s) {
    double *d_h = reinterpret_cast<double *>(b.params);
    double *d_k = reinterpret_cast<double *>(b.params + h.o_k);
    double *d_kh = reinterpret_cast<double *>(b.params + h.o_kh);
    if (!h.inline_params) {
        P2P_TRY(no_capture(s, "a Helmholtz set-up that uploads its parameters"));
        std::vector<char> hp(h.param_bytes);
        for (int32_t g = 0; g < h.n_grids; ++g) {
            std::memcpy(hp.data() + 8 * g, &grids[g].h, 8);
            std::memcpy(hp.data() + h.o_k + 8 * g, &grids[g].k, 8);
        }
        std::memcpy(hp.data() + h.o_kh, h.khs.data(), 8 * static_cast<size_t>(h.n_tables));
        std::memcpy(hp.data() + h.o_itab, h.itab.data(), 4 * static_cast<size_t>(h.n_grids));
        std::memcpy(hp.data() + h.o_isc, h.iscale.data(), 4 * static_cast<size_t>(h.n_grids));
        if (h.cols) helmholtz_cols_tiles(grids, h.n_grids, reinterpret_cast<int32_t *>(hp.data() + h.o_tiles));
        // a copy from pageable memory has read its source when it returns
        P2P_HIP(hipMemcpyAsync(b.params, hp.data(), h.param_bytes, hipMemcpyHostToDevice, s));
    }
    if (h.blk) P2P_TRY(launch_green_blocks(d_kh, h.inl, h.n_tables, h.copies, h.cols, h.fp64, b.blocks, s));
    else P2P_TRY(launch_green_tables(d_h, d_k, h.n_grids, h.fp64, b.table, s));
    return P2P_OK;
}

// Argument checks of an evaluation that come after the workspace query.
p2p_status helm_check_call(const HelmSetup &h, const p2p_tree *tree, const p2p_nbrs *nbrs,
                           const p2p_redundant *red, p2p_layout layout, const void *q, void *u, int32_t conj) {
    const bool redundant = layout == P2P_REDUNDANT;
    const int64_t n = tree->n;
    const int32_t nrhs = h.nrhs;
    if (n > 0 && !u) return fail(P2P_EINVAL, "u must not be NULL");
    if (redundant) {
        if (!red) return fail(P2P_EINVAL, "REDUNDANT layout needs red");
        if (red->kind != P2P_KIND_HELMHOLTZ) return fail(P2P_EINVAL, "red was not built for Helmholtz");
        if ((red->prec == P2P_FP64) != h.fp64) return fail(P2P_EINVAL, "red was built with another payload precision");
        if (red->nrhs != nrhs) return fail(P2P_EINVAL, "red was built with another nrhs");
        if (!red->red_start || (red->count > 0 && !red->planes[0])) return fail(P2P_EINVAL, "red arrays must not be NULL");
        if (red->grain != 0 && red->grain != 1 && red->grain != 2 && red->grain != 4)
            return fail(P2P_EINVAL, "red->grain must be 0, 1, 2 or 4");
        if (red->grain > 1 && nbrs->count > 0 && !red->red_row)
            return fail(P2P_EINVAL, "a tile-grain layout needs red->red_row");
        if (conj) return fail(P2P_EUNSUPPORTED, "conjugated action needs the GATHER layout");
    } else if (n > 0 && !q) {
        return fail(P2P_EINVAL, "q must not be NULL");
    }
    return P2P_OK;
}

// The evaluation from a filled set-up: the sorted copy of q (GATHER), then one
// product launch (the matrix-core queues' counters are zeroed first; one RHS on a
// grid of few tiles adds the join of the two halves of each tile).
p2p_status helm_run(const HelmSetup &h, const HelmSetupBufs &b, int32_t *counter, char *sorted, double2 *parts,
                    const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red, p2p_layout layout,
                    const void *q, void *u, int32_t conj, hipStream_t s) {
    P2P_TRY(helm_check_call(h, tree, nbrs, red, layout, q, u, conj));
    const bool redundant = layout == P2P_REDUNDANT;
    const int64_t n = tree->n, L = tree->n_leaves;
    const int32_t nrhs = h.nrhs;
    const bool tiled = redundant && red->grain > 1;
    if (!redundant) {
        if (h.fp64)
            P2P_TRY(launch_permute_rows<double2>(static_cast<const double2 *>(q), tree->perm, n, nrhs,
                                                 reinterpret_cast<double2 *>(sorted), s));
        else
            P2P_TRY(launch_permute_rows<float2>(static_cast<const float2 *>(q), tree->perm, n, nrhs,
                                                reinterpret_cast<float2 *>(sorted), s));
    }
    const int32_t *d_itab = reinterpret_cast<const int32_t *>(b.params + h.o_itab);
    const float *d_iscale = reinterpret_cast<const float *>(b.params + h.o_isc);
    const int32_t *d_tiles = reinterpret_cast<const int32_t *>(b.params + h.o_tiles);
    if (h.cols || h.mfma) {
        HelmholtzMfmaArgs a{};
        a.L = L;
        a.key_bits = tree->key_bits;
        a.leaf_start = tree->leaf_start;
        a.leaf_key = tree->leaf_key;
        a.perm = tree->perm;
        a.nbr_start = nbrs->nbr_start;
        a.nbr_idx = nbrs->nbr_idx;
        a.red_start = redundant ? red->red_start : nullptr;
        a.red_row = tiled ? red->red_row : nullptr;
        a.src = redundant ? static_cast<const float2 *>(red->planes[0]) : reinterpret_cast<const float2 *>(sorted);
        a.blocks = b.blocks;
        const int64_t nblk = static_cast<int64_t>(h.n_tables) * 27 * 4096;
        a.zeros = !h.cols ? nullptr
                  : h.fp64 ? reinterpret_cast<const float2 *>(reinterpret_cast<const double2 *>(b.blocks) + nblk)
                           : b.blocks + nblk;
        a.inst_h = h.inline_params ? nullptr : reinterpret_cast<const double *>(b.params);
        a.n = n;
        a.parts = parts;
        a.inst_table = d_itab;
        a.inst_scale = d_iscale;
        a.conj = conj;
        a.comp = h.prec == P2P_FP32_MIXED;
        a.u = static_cast<float2 *>(u);
        if (h.cols) {
            a.copies = 1;
            a.nrhs = 1;
            return launch_helmholtz_mfma_cols(a, d_tiles, h.inl, h.n_tiles, redundant, h.fp64, s);
        }
        a.copies = h.copies;
        a.counter = counter;
        a.nrhs = nrhs;
        return launch_helmholtz_mfma(a, redundant, h.waves_per_wg, h.wg_per_cu, h.rhs_tile, s);
    }
    HelmholtzArgs a{};
    a.L = L;
    a.key_bits = tree->key_bits;
    a.leaf_start = tree->leaf_start;
    a.leaf_key = tree->leaf_key;
    a.perm = tree->perm;
    a.nbr_start = nbrs->nbr_start;
    a.nbr_idx = nbrs->nbr_idx;
    a.red_start = redundant ? red->red_start : nullptr;
    a.red_row = tiled ? red->red_row : nullptr;
    a.src = redundant ? red->planes[0] : sorted;
    a.table = b.table;
    a.nrhs = nrhs;
    a.conj = conj;
    a.comp = h.prec == P2P_FP32_MIXED;
    a.u = u;
    return launch_helmholtz(a, redundant, h.fp64, s);
}

// Per-call scratch of an evaluation beside the set-up: the eight queue counters
// (matrix cores, several RHS), the sorted copy of q (GATHER) and, for one RHS,
// the two partial results of tiles whose offsets two workgroups share.
void helm_take_call(Arena &ar, const HelmSetup &h, int64_t n, bool redundant, int32_t **counter, char **sorted,
                    double2 **parts) {
    const size_t csize = h.fp64 ? sizeof(double2) : sizeof(float2);
    *counter = h.mfma ? ar.take<int32_t>(64) : nullptr;
    *sorted = redundant ? nullptr : ar.take<char>(static_cast<size_t>(n) * h.nrhs * csize);
    *parts = h.cols ? ar.take<double2>(2 * static_cast<size_t>(n)) : nullptr;
}

p2p_status helmholtz_common(const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_redundant *red,
                            p2p_layout layout, p2p_precision prec, const p2p_grid *grids,
                            int32_t n_grids, int32_t nrhs, const void *q, void *u, int32_t conj,
                            const int32_t *tile, void *ws, size_t *ws_bytes, hipStream_t s) {
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    HelmSetup h;
    P2P_TRY(helm_setup(tree, nbrs, prec, grids, n_grids, nrhs, tile, &h));
    if (layout != P2P_GATHER && layout != P2P_REDUNDANT) return fail(P2P_EINVAL, "bad layout");
    Arena ar(ws);
    const HelmSetupBufs b = helm_take(ar, h);
    int32_t *counter;
    char *sorted;
    double2 *parts;
    helm_take_call(ar, h, tree->n, layout == P2P_REDUNDANT, &counter, &sorted, &parts);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    // every argument is checked before the set-up is queued
    P2P_TRY(helm_check_call(h, tree, nbrs, red, layout, q, u, conj));
    P2P_TRY(helm_fill(h, b, tree, nbrs, grids, s));
    return helm_run(h, b, counter, sorted, parts, tree, nbrs, red, layout, q, u, conj, s);
}

// FNV-1a over the arguments a set-up depends on.
struct Fnv {
    uint64_t v = 1469598103934665603ull;
    template <class T>
    void add(const T &x) {
        const unsigned char *p = reinterpret_cast<const unsigned char *>(&x);
        for (size_t i = 0; i < sizeof(T); ++i) {
            v ^= p[i];
            v *= 1099511628211ull;
        }
    }
};

uint64_t helm_fingerprint(const HelmSetup &h, const p2p_tree *tree, const p2p_nbrs *nbrs, const p2p_grid *grids) {
    Fnv f;
    f.add(tree->n);
    f.add(tree->n_leaves);
    f.add(tree->key_bits);
    f.add(nbrs->count);
    f.add(static_cast<int32_t>(h.prec));
    f.add(h.nrhs);
    f.add(h.waves_per_wg);
    f.add(h.wg_per_cu);
    f.add(h.rhs_tile);
    f.add(h.copies);
    f.add(h.n_grids);
    for (int32_t g = 0; g < h.n_grids; ++g) {
        f.add(grids[g].n_side);
        f.add(grids[g].h);
        f.add(grids[g].k);
        f.add(grids[g].point_off);
    }
    return f.v == 0 ? 1 : f.v;
}

}  // namespace

extern "C" p2p_status p2p_eval_helmholtz(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                         const p2p_redundant *red, p2p_layout layout,
                                         p2p_precision prec, const p2p_grid *grids, int32_t n_grids,
                                         int32_t nrhs, const void *q, void *u, const int32_t *tile,
                                         void *ws, size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    return helmholtz_common(tree, nbrs, red, layout, prec, grids, n_grids, nrhs, q, u, 0, tile, ws,
                            ws_bytes, as_stream(stream));
}

extern "C" p2p_status p2p_helmholtz_prepare(const p2p_tree *tree, const p2p_nbrs *nbrs, p2p_precision prec,
                                            const p2p_grid *grids, int32_t n_grids, int32_t nrhs,
                                            const int32_t *tile, p2p_helmholtz_plan *plan,
                                            p2p_stream_t stream) {
    set_error("");
    if (!plan) return fail(P2P_EINVAL, "plan is NULL");
    HelmSetup h;
    P2P_TRY(helm_setup(tree, nbrs, prec, grids, n_grids, nrhs, tile, &h));
    Arena ar(plan->buf);
    const HelmSetupBufs b = helm_take(ar, h);
    if (!plan->buf) {
        plan->bytes = ar.used;
        return P2P_OK;
    }
    if (plan->bytes < ar.used)
        return fail(P2P_EINVAL, "plan->bytes too small: need " + std::to_string(ar.used) + ", got " +
                                    std::to_string(plan->bytes));
    if ((reinterpret_cast<uintptr_t>(plan->buf) & 255u) != 0) return fail(P2P_EINVAL, "plan->buf must be 256-byte aligned");
    P2P_TRY(helm_fill(h, b, tree, nbrs, grids, as_stream(stream)));
    plan->prec = prec;
    plan->nrhs = nrhs;
    plan->tile[0] = h.waves_per_wg;
    plan->tile[1] = h.wg_per_cu;
    plan->tile[2] = h.rhs_tile;
    plan->tile[3] = h.copies;
    plan->tiled = tile ? 1 : 0;
    plan->fingerprint = helm_fingerprint(h, tree, nbrs, grids);
    return P2P_OK;
}

extern "C" p2p_status p2p_eval_helmholtz_prepared(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                                  const p2p_redundant *red, p2p_layout layout,
                                                  const p2p_grid *grids, int32_t n_grids,
                                                  const p2p_helmholtz_plan *plan, const void *q, void *u,
                                                  void *ws, size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    if (!plan || !plan->buf || plan->fingerprint == 0) return fail(P2P_EINVAL, "plan was not prepared");
    if (layout != P2P_GATHER && layout != P2P_REDUNDANT) return fail(P2P_EINVAL, "bad layout");
    HelmSetup h;
    P2P_TRY(helm_setup(tree, nbrs, static_cast<p2p_precision>(plan->prec), grids, n_grids, plan->nrhs,
                       plan->tiled ? plan->tile : nullptr, &h));
    if (helm_fingerprint(h, tree, nbrs, grids) != plan->fingerprint)
        return fail(P2P_EINVAL, "plan was prepared for another tree, grid set, precision, nrhs or tile");
    Arena pa(plan->buf);
    const HelmSetupBufs b = helm_take(pa, h);
    if (plan->bytes < pa.used) return fail(P2P_EINVAL, "plan->bytes smaller than the set-up");
    Arena ar(ws);
    int32_t *counter;
    char *sorted;
    double2 *parts;
    helm_take_call(ar, h, tree->n, layout == P2P_REDUNDANT, &counter, &sorted, &parts);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    return helm_run(h, b, counter, sorted, parts, tree, nbrs, red, layout, q, u, 0, as_stream(stream));
}

// ------------------------------------------------------------- adjoint ----
extern "C" p2p_status p2p_adjoint(int32_t kind, const p2p_tree *tree, const p2p_nbrs *nbrs,
                                  const p2p_redundant *red, p2p_layout layout, p2p_precision prec,
                                  double eps, const p2p_grid *grids, int32_t n_grids, int32_t nrhs,
                                  int32_t conjugate, const void *const fwd_in[4],
                                  const void *const grad_out[4], void *const grad_in[4], void *ws,
                                  size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    hipStream_t s = as_stream(stream);
    if (kind == P2P_KIND_HELMHOLTZ) {
        if (layout != P2P_GATHER) return fail(P2P_EUNSUPPORTED, "Helmholtz adjoint uses the GATHER layout");
        if (conjugate != 0 && conjugate != 1) return fail(P2P_EINVAL, "conjugate must be 0 or 1");
        const void *g = grad_out ? grad_out[0] : nullptr;
        void *out = grad_in ? grad_in[0] : nullptr;
        // A is symmetric (reciprocity and a symmetric near relation): A^T g = A g
        return helmholtz_common(tree, nbrs, red, P2P_GATHER, prec, grids, n_grids, nrhs, g, out,
                                conjugate, nullptr, ws, ws_bytes, s);
    }
    if (kind != P2P_KIND_GRAVITY) return fail(P2P_EINVAL, "kind must be P2P_KIND_GRAVITY or P2P_KIND_HELMHOLTZ");
    (void)red;
    P2P_TRY(check_tree(tree));
    if (tree->kind != P2P_TREE_PARTICLES) return fail(P2P_EINVAL, "gravity needs a particle tree");
    P2P_TRY(check_nbrs(tree, nbrs));
    if (layout != P2P_GATHER) return fail(P2P_EUNSUPPORTED, "gravity adjoint uses the GATHER layout");
    P2P_TRY(check_gravity_prec(prec));
    P2P_TRY(check_eps(eps, prec == P2P_FP32_MIXED, true));
    const int64_t n = tree->n;
    Arena ar(ws);
    Row4d *s4 = ar.take<Row4d>(n);
    Row4d *g4 = ar.take<Row4d>(n);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (!fwd_in || !grad_out || !grad_in) return fail(P2P_EINVAL, "fwd_in, grad_out, grad_in must not be NULL");
    for (int i = 0; i < 4; ++i)
        if (n > 0 && (!fwd_in[i] || !grad_out[i] || !grad_in[i])) return fail(P2P_EINVAL, "NULL gravity array");
    auto D = [](const void *p) { return static_cast<const double *>(p); };
    P2P_TRY(launch_scatter4(D(fwd_in[0]), D(fwd_in[1]), D(fwd_in[2]), D(fwd_in[3]), tree->iperm, n, s4, s));
    P2P_TRY(launch_scatter4(D(grad_out[0]), D(grad_out[1]), D(grad_out[2]), D(grad_out[3]), tree->iperm, n,
                            g4, s));
    GravityAdjointArgs a{};
    a.L = tree->n_leaves;
    a.leaf_start = tree->leaf_start;
    a.perm = tree->perm;
    a.nbr_start = nbrs->nbr_start;
    a.nbr_idx = nbrs->nbr_idx;
    a.nbr_shift = shifts(nbrs);
    a.s4 = s4;
    a.g4 = g4;
    a.leaf_key = tree->leaf_key;
    a.leaf_level = tree->leaf_level;
    a.eps2 = eps * eps;
    a.gx = static_cast<double *>(grad_in[0]);
    a.gy = static_cast<double *>(grad_in[1]);
    a.gz = static_cast<double *>(grad_in[2]);
    a.gm = static_cast<double *>(grad_in[3]);
    return launch_gravity_adjoint(a, prec == P2P_FP32_MIXED, s);
}

// ------------------------------------------------------------ Locality ----
extern "C" p2p_status p2p_locality(const p2p_tree *tree, const p2p_nbrs *nbrs,
                                   const p2p_redundant *red, double bytes_per_entry,
                                   double cache_bytes, p2p_locality_t *out, void *ws,
                                   size_t *ws_bytes, p2p_stream_t stream) {
    set_error("");
    if (!ws_bytes) return fail(P2P_EINVAL, "ws_bytes must not be NULL");
    P2P_TRY(check_tree(tree));
    P2P_TRY(check_nbrs(tree, nbrs));
    if (!(bytes_per_entry > 0.0) || !(cache_bytes > 0.0)) return fail(P2P_EINVAL, "bytes_per_entry and cache_bytes must be > 0");
    Arena ar(ws);
    unsigned long long *sums = ar.take<unsigned long long>(3);
    p2p_status st;
    if (ws_query(ws, ws_bytes, ar, &st)) return st;
    if (!out) return fail(P2P_EINVAL, "out is NULL");
    hipStream_t s = as_stream(stream);
    P2P_TRY(no_capture(s, "p2p_locality"));
    const int64_t L = tree->n_leaves;
    P2P_HIP(hipMemsetAsync(sums, 0, 3 * sizeof(unsigned long long), s));
    P2P_TRY(launch_locality_stats(tree->leaf_start, nbrs->nbr_start, nbrs->nbr_idx, L, sums, s));
    unsigned long long h[3] = {0, 0, 0};
    P2P_HIP(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
    const int64_t S = red ? red->count : static_cast<int64_t>(h[1]);
    out->entries = S;
    out->pairs = static_cast<int64_t>(h[2]) - tree->n;
    out->d_mean = L > 0 ? static_cast<double>(h[0]) / static_cast<double>(L) : 0.0;
    out->v_gather = static_cast<double>(tree->n) * bytes_per_entry;
    out->v_red = static_cast<double>(S) * bytes_per_entry;
    out->d_ratio = out->d_mean / 1.0;
    out->v_ratio = out->v_red > 0 ? out->v_gather / out->v_red : 0.0;
    out->locality = (out->v_red <= cache_bytes) ? out->d_ratio * out->v_ratio
                                                : (out->d_ratio > 0 ? out->v_ratio / out->d_ratio : 0.0);
    return P2P_OK;
}
