// Near-field lists (the E2 neighbourhood, Sec. 5.1): for every leaf A, every leaf B whose closed cube
// touches A's, A included, in ascending leaf id.
//
// One wavefront per leaf.  Lanes 0..26 each take one of the 27 cells of A's
// size around A (A itself in the middle).  A leaf touching A either covers
// such a cell (it is at least as large as A) or lies inside one.  Each lane
// finds, by binary search over the sorted leaf keys, the contiguous range of
// leaves that meet its cell.  The ranges of different cells are disjoint,
// except that one large leaf may cover several cells; those duplicates are
// dropped and the ranges are put in key order, which is leaf-id order.  The
// candidates are then tested in parallel, 64 per step, and the adjacent ones
// written with a ballot prefix, so the list comes out ascending.
//
// The counting pass (counts != NULL) also sums, per leaf A, the points of the
// leaves in nbr(A): the length of A's segment in the redundant layout.
//
// The searches start from a directory over the top bits of the key: dir[p]
// is the first leaf whose key is at least p << shift, so a key's bucket bounds
// its search to the leaves of that bucket.
//
// Periodic lists (particles on the unit torus): a cell past a face of the
// domain wraps to the opposite side and carries the image code of that wrap,
// c = (sx+1) + 3 (sy+1) + 9 (sz+1); its leaves are tested shifted by
// (sx, sy, sz) domain edges.  Ranges are deduplicated and ordered by (c, lo),
// so the list comes out ascending in (c, B); one leaf may appear under
// several codes.
#include "p2p_internal.h"

namespace p2p {
namespace {

constexpr int kNbrWaves = 4;
constexpr int kNbrSlots = kNbrSlotsPerLeaf;

// First index in [lo, hi) with a[i] > v (upper) or a[i] >= v (lower).
__device__ inline int64_t bound_in(const uint64_t *__restrict__ a, int64_t lo, int64_t hi, uint64_t v,
                                   bool upper) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (upper ? (a[mid] <= v) : (a[mid] < v)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int64_t dir_bound(const uint64_t *__restrict__ a, const int32_t *__restrict__ dir,
                                    int dir_bits, int shift, uint64_t v, bool upper) {
    const uint64_t p = v >> shift;
    if (p >= (1ull << dir_bits)) return dir[1ull << dir_bits];
    return bound_in(a, dir[p], dir[p + 1], v, upper);
}

// Also clears the two counters of the counting pass that follows (lists over
// kNbrSlots entries, heavy leaves).
__global__ void k_key_directory(const uint64_t *__restrict__ leaf_key, int64_t L, int dir_bits,
                                int shift, int32_t *__restrict__ dir, int32_t *__restrict__ counters) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t(1) << dir_bits) + 1;
    if (p == 0) {
        counters[0] = 0;
        counters[1] = 0;
    }
    if (p >= nb) return;
    dir[p] = (p == nb - 1) ? static_cast<int32_t>(L)
                           : static_cast<int32_t>(bound_in(leaf_key, 0, L, static_cast<uint64_t>(p) << shift, false));
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// COUNT: counts[A], segs[A], the first kNbrSlots entries of nbr(A) into
// slots[A * kNbrSlots ...], and +1 on counters[0] for a longer list.
// FILL: nbr(A) into nbr_idx[nbr_start[A] ...], only for leaves whose list
// did not fit its slots (counts[A] > kNbrSlots).
enum { kNbrCount = 0, kNbrFill = 1 };

// A leaf with more candidates than this (a large leaf beside a finely split
// region) is left to k_neighbors_heavy, which spreads its candidates over a
// whole workgroup; in one wavefront it would set the time of the whole pass.
constexpr int32_t kHeavyCands = 1024;
constexpr int kHeavyWaves = 16;
constexpr unsigned kHeavyGrid = 512;

// What one leaf's search needs: the candidate (source) tree's arrays and key
// directory, the target leaves' keys and levels (the same tree for plain
// lists, another one for remote lists), and the key layout.
struct NbrTree {
    const uint64_t *leaf_key;
    const int8_t *leaf_level;
    const int32_t *leaf_start;
    const int32_t *dir;
    int64_t L;
    const uint64_t *tkey;
    const int8_t *tlevel;
    int64_t Lt;
    int key_bits, inst_shift, dir_bits, dir_shift;
};

// Leaf A's geometry in key units: anchor a, edge sA.
struct NbrLeaf {
    int64_t a[3];
    int64_t sA, dim;
    uint64_t local_mask, inst_bits;
    int lA;
};

__device__ inline NbrLeaf nbr_leaf(const NbrTree &t, int64_t A) {
    NbrLeaf f;
    const uint64_t kA = t.tkey[A];
    f.lA = t.tlevel[A];
    f.dim = int64_t(1) << t.key_bits;
    f.sA = int64_t(1) << (t.key_bits - f.lA);
    f.local_mask = (3 * t.key_bits >= 64) ? ~0ull : ((1ull << (3 * t.key_bits)) - 1ull);
    f.inst_bits = (t.inst_shift >= 64) ? 0ull : (kA >> t.inst_shift) << t.inst_shift;
    const uint64_t local = kA & f.local_mask;
    f.a[0] = p2pd::compact3(local);
    f.a[1] = p2pd::compact3(local >> 1);
    f.a[2] = p2pd::compact3(local >> 2);
    return f;
}

// Called by one whole wavefront: the candidate ranges of leaf A in (code, lo)
// order into s_lo[0..K), their exclusive prefix into s_pre[0..K] and, with
// PER, their image codes into s_code.  Returns the candidate total; K in *Kout.
template <bool PER>
__device__ int32_t nbr_ranges(const NbrTree &t, const NbrLeaf &f, int32_t *s_lo, int32_t *s_pre,
                              int32_t *s_code, int *Kout) {
    const int lane = threadIdx.x & 63;
    // ---- one cell per lane
    int64_t lo = 0, hi = 0;
    bool valid = false;
    int code = 13;
    if (lane < 27) {
        int64_t c[3] = {f.a[0] + (lane % 3 - 1) * f.sA, f.a[1] + ((lane / 3) % 3 - 1) * f.sA,
                        f.a[2] + (lane / 9 - 1) * f.sA};
        bool inside = c[0] >= 0 && c[1] >= 0 && c[2] >= 0 && c[0] < f.dim && c[1] < f.dim && c[2] < f.dim;
        if constexpr (PER) {
            // c lies in [-sA, dim + sA) with sA <= dim: one wrap per axis
            int wrap[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                wrap[d] = c[d] < 0 ? -1 : (c[d] >= f.dim ? 1 : 0);
                c[d] -= wrap[d] * f.dim;
            }
            code = (wrap[0] + 1) + 3 * (wrap[1] + 1) + 9 * (wrap[2] + 1);
            inside = true;
        }
        if (inside) {
            const uint64_t kC = f.inst_bits | p2pd::morton3(static_cast<uint32_t>(c[0]),
                                                            static_cast<uint32_t>(c[1]),
                                                            static_cast<uint32_t>(c[2]));
            const uint64_t sizeC = 1ull << (3 * (t.key_bits - f.lA));
            const int64_t j = dir_bound(t.leaf_key, t.dir, t.dir_bits, t.dir_shift, kC, true) - 1;
            bool covers = false;
            if (j >= 0) {
                const uint64_t sj = 1ull << (3 * (t.key_bits - t.leaf_level[j]));
                covers = kC < t.leaf_key[j] + sj;   // leaf_key[j] <= kC by construction
            }
            lo = covers ? j : j + 1;
            // a covering leaf at least as large as the cell holds all of it
            // (aligned cubes); only a cell split into smaller leaves needs
            // the search for its end
            if (covers && t.leaf_level[j] <= f.lA)
                hi = j + 1;
            else
                hi = dir_bound(t.leaf_key, t.dir, t.dir_bits, t.dir_shift, kC + sizeC, false);
            valid = lo < hi;
        }
    }
    // ---- drop duplicate ranges (one large leaf covering several cells of
    // one image), rank by (code, lo); the loops stay rolled (fully unrolled,
    // their shuffles would hold enough registers to halve the occupancy of a
    // search that is bound by load latency)
    bool first = valid;
#pragma unroll 1
    for (int q = 0; q < 27; ++q) {
        const int64_t loq = __shfl(lo, q, 64);
        const int vq = __shfl(static_cast<int>(valid), q, 64);
        const int cq = PER ? __shfl(code, q, 64) : 13;
        if (vq && q < lane && loq == lo && cq == code) first = false;
    }
    int rank = 0;
#pragma unroll 1
    for (int q = 0; q < 27; ++q) {
        const int64_t loq = __shfl(lo, q, 64);
        const int fq = __shfl(static_cast<int>(first), q, 64);
        const int cq = PER ? __shfl(code, q, 64) : 13;
        if (fq && (cq < code || (cq == code && loq < lo))) ++rank;
    }
    const int K = __popcll(__ballot(first));
    if (first) {
        s_lo[rank] = static_cast<int32_t>(lo);
        s_pre[rank] = static_cast<int32_t>(hi - lo);
        if constexpr (PER) s_code[rank] = code;
    }
    wave_sync();
    // exclusive prefix of the range lengths in sorted order
    int32_t len = (lane < K) ? s_pre[lane] : 0;
    int32_t inc = len;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
        int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    wave_sync();
    if (lane < K) s_pre[lane] = inc - len;
    const int32_t total = __shfl(inc, K > 0 ? K - 1 : 0, 64);
    if (lane == 0) s_pre[K] = total;
    wave_sync();
    *Kout = K;
    return total;
}

// Candidate cidx (< total) of the ranges: leaf B, image code cB, and whether
// B (shifted by its image) touches A.
template <bool PER>
__device__ inline bool nbr_candidate(const NbrTree &t, const NbrLeaf &f, int32_t cidx, int K,
                                     const int32_t *s_lo, const int32_t *s_pre, const int32_t *s_code,
                                     int64_t &B, int &cB) {
    int r = 0;
    while (r + 1 < K && s_pre[r + 1] <= cidx) ++r;
    B = s_lo[r] + (cidx - s_pre[r]);
    cB = PER ? s_code[r] : 13;
    const uint64_t kB = t.leaf_key[B] & f.local_mask;
    const int64_t sB = int64_t(1) << (t.key_bits - t.leaf_level[B]);
    int64_t b[3] = {p2pd::compact3(kB), p2pd::compact3(kB >> 1), p2pd::compact3(kB >> 2)};
    if constexpr (PER) {
        b[0] += (cB % 3 - 1) * f.dim;
        b[1] += ((cB / 3) % 3 - 1) * f.dim;
        b[2] += (cB / 9 - 1) * f.dim;
    }
    bool adj = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) adj = adj && (f.a[d] <= b[d] + sB) && (b[d] <= f.a[d] + f.sA);
    return adj;
}

// Writes one adjacent candidate at list position pos (COUNT: into the slots if
// it is among the first kNbrSlots; FILL: into the CSR list).
template <int MODE, bool PER>
__device__ inline void nbr_put(int64_t A, int64_t pos, int64_t out0, int64_t B, int cB, int32_t *slots,
                               int8_t *slot_code, int32_t *nbr_idx, int8_t *nbr_shift) {
    if (MODE == kNbrFill) {
        nbr_idx[out0 + pos] = static_cast<int32_t>(B);
        if constexpr (PER) nbr_shift[out0 + pos] = static_cast<int8_t>(cB);
    } else if (pos < kNbrSlots) {
        slots[A * kNbrSlots + pos] = static_cast<int32_t>(B);
        if constexpr (PER) slot_code[A * kNbrSlots + pos] = static_cast<int8_t>(cB);
    }
}

// One wavefront per leaf; a leaf with more than kHeavyCands candidates is
// appended to heavy[] (COUNT) or skipped (FILL) for k_neighbors_heavy.
// PER: periodic lists; slot_code / nbr_shift receive the image codes.
template <int MODE, bool PER>
__global__ __launch_bounds__(64 * kNbrWaves) void k_neighbors(
    NbrTree t, int32_t *__restrict__ counts, int32_t *__restrict__ segs, int32_t *__restrict__ slots,
    int8_t *__restrict__ slot_code, int32_t *__restrict__ counters, int32_t *__restrict__ heavy,
    const int64_t *__restrict__ nbr_start, int32_t *__restrict__ nbr_idx, int8_t *__restrict__ nbr_shift) {
    __shared__ int32_t s_lo[kNbrWaves][32];
    __shared__ int32_t s_pre[kNbrWaves][33];
    __shared__ int32_t s_code[kNbrWaves][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t A = static_cast<int64_t>(blockIdx.x) * kNbrWaves + w;
    if (A >= t.Lt) return;
    if (MODE == kNbrFill && counts[A] <= kNbrSlots) return;
    const NbrLeaf f = nbr_leaf(t, A);
    int K = 0;
    const int32_t total = nbr_ranges<PER>(t, f, s_lo[w], s_pre[w], s_code[w], &K);
    if (total > kHeavyCands) {
        if (MODE == kNbrCount && lane == 0) heavy[atomicAdd(&counters[1], 1)] = static_cast<int32_t>(A);
        return;
    }

    // ---- test candidates, 64 at a time, in ascending (code, leaf id)
    const int64_t out0 = (MODE == kNbrFill) ? nbr_start[A] : 0;
    int64_t written = 0;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int32_t occ_sum = 0;     // points of this lane's adjacent candidates (count pass)
    for (int32_t base = 0; base < total; base += 64) {
        const int32_t cidx = base + lane;
        bool adj = false;
        int64_t B = 0;
        int cB = 13;
        if (cidx < total) adj = nbr_candidate<PER>(t, f, cidx, K, s_lo[w], s_pre[w], s_code[w], B, cB);
        const uint64_t bal = __ballot(adj);
        const int64_t pos = written + __popcll(bal & below);
        if (adj) {
            nbr_put<MODE, PER>(A, pos, out0, B, cB, slots, slot_code, nbr_idx, nbr_shift);
            if (MODE == kNbrCount) occ_sum += t.leaf_start[B + 1] - t.leaf_start[B];
        }
        written += __popcll(bal);
    }
    if (MODE == kNbrCount) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) occ_sum += __shfl_xor(occ_sum, o, 64);
        if (lane == 0) {
            counts[A] = static_cast<int32_t>(written);
            segs[A] = occ_sum;
            if (written > kNbrSlots) atomicAdd(&counters[0], 1);
        }
    }
}

// The leaves heavy[0 .. counters[1]), one workgroup each (grid-stride): the
// first wavefront finds the ranges, the candidates are split into
// kHeavyWaves contiguous runs, one per wavefront; a first sweep counts each
// run's adjacent candidates, their prefix gives each run its first list
// position, and a second sweep writes the entries (COUNT: only runs that
// reach into the first kNbrSlots positions).
template <int MODE, bool PER>
__global__ __launch_bounds__(64 * kHeavyWaves) void k_neighbors_heavy(
    NbrTree t, int32_t *__restrict__ counts, int32_t *__restrict__ segs, int32_t *__restrict__ slots,
    int8_t *__restrict__ slot_code, int32_t *__restrict__ counters, const int32_t *__restrict__ heavy,
    const int64_t *__restrict__ nbr_start, int32_t *__restrict__ nbr_idx, int8_t *__restrict__ nbr_shift) {
    __shared__ int32_t s_lo[32];
    __shared__ int32_t s_pre[33];
    __shared__ int32_t s_code[32];
    __shared__ int32_t s_meta[2];                 // K, total
    __shared__ int32_t s_cnt[kHeavyWaves];        // adjacent candidates per run
    __shared__ int32_t s_occ[kHeavyWaves];        // their points (COUNT)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t nh = counters[1];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int32_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const int64_t A = heavy[h];
        if (MODE == kNbrFill && counts[A] <= kNbrSlots) continue;   // uniform over the block
        const NbrLeaf f = nbr_leaf(t, A);
        if (w == 0) {
            int K = 0;
            const int32_t total = nbr_ranges<PER>(t, f, s_lo, s_pre, s_code, &K);
            if (lane == 0) {
                s_meta[0] = K;
                s_meta[1] = total;
            }
        }
        __syncthreads();
        const int K = s_meta[0];
        const int32_t total = s_meta[1];
        const int32_t run = (total + kHeavyWaves - 1) / kHeavyWaves;
        const int32_t c0 = min(total, w * run), c1 = min(total, c0 + run);
        // first sweep: count
        int32_t cnt = 0, occ_sum = 0;
        for (int32_t base = c0; base < c1; base += 64) {
            const int32_t cidx = base + lane;
            bool adj = false;
            int64_t B = 0;
            int cB = 13;
            if (cidx < c1) adj = nbr_candidate<PER>(t, f, cidx, K, s_lo, s_pre, s_code, B, cB);
            cnt += __popcll(__ballot(adj));
            if (MODE == kNbrCount && adj) occ_sum += t.leaf_start[B + 1] - t.leaf_start[B];
        }
        if (MODE == kNbrCount) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) occ_sum += __shfl_xor(occ_sum, o, 64);
        }
        if (lane == 0) {
            s_cnt[w] = cnt;
            s_occ[w] = occ_sum;
        }
        __syncthreads();
        int64_t first = 0, all = 0, occ_all = 0;
        for (int q = 0; q < kHeavyWaves; ++q) {
            if (q < w) first += s_cnt[q];
            all += s_cnt[q];
            occ_all += s_occ[q];
        }
        // second sweep: write
        if (MODE == kNbrFill || first < kNbrSlots) {
            const int64_t out0 = (MODE == kNbrFill) ? nbr_start[A] : 0;
            int64_t written = first;
            for (int32_t base = c0; base < c1; base += 64) {
                if (MODE == kNbrCount && written >= kNbrSlots) break;   // uniform
                const int32_t cidx = base + lane;
                bool adj = false;
                int64_t B = 0;
                int cB = 13;
                if (cidx < c1) adj = nbr_candidate<PER>(t, f, cidx, K, s_lo, s_pre, s_code, B, cB);
                const uint64_t bal = __ballot(adj);
                const int64_t pos = written + __popcll(bal & below);
                if (adj) nbr_put<MODE, PER>(A, pos, out0, B, cB, slots, slot_code, nbr_idx, nbr_shift);
                written += __popcll(bal);
            }
        }
        if (MODE == kNbrCount && threadIdx.x == 0) {
            counts[A] = static_cast<int32_t>(all);
            segs[A] = static_cast<int32_t>(occ_all);
            if (all > kNbrSlots) atomicAdd(&counters[0], 1);
        }
        __syncthreads();   // the LDS ranges are rewritten for the next leaf
    }
}

// Slots into the CSR lists: thread (A, s) moves entry s of a list that fit
// (and its image code, if slot_code is not null).
__global__ void k_compact_slots(const int32_t *__restrict__ counts, const int32_t *__restrict__ slots,
                                const int8_t *__restrict__ slot_code,
                                const int64_t *__restrict__ nbr_start, int64_t L,
                                int32_t *__restrict__ nbr_idx, int8_t *__restrict__ nbr_shift) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t A = t / kNbrSlots;
    const int sidx = static_cast<int>(t % kNbrSlots);
    if (A >= L) return;
    const int32_t c = counts[A];
    if (c <= kNbrSlots && sidx < c) {
        nbr_idx[nbr_start[A] + sidx] = slots[t];
        if (slot_code) nbr_shift[nbr_start[A] + sidx] = slot_code[t];
    }
}

// The list totals E and S and the number of overflowing lists, gathered for
// one read-back.
__global__ void k_nbr_totals(const int64_t *__restrict__ start, const int64_t *__restrict__ seg_scan,
                             const int32_t *__restrict__ counters, int64_t L, int64_t *__restrict__ out) {
    out[0] = L > 0 ? start[L] : 0;
    out[1] = L > 0 ? seg_scan[L] : 0;
    out[2] = counters[0];
}

}  // namespace

int neighbor_dir_bits(int total_key_bits) { return total_key_bits < 18 ? total_key_bits : 18; }

p2p_status launch_key_directory(const uint64_t *leaf_key, int64_t L, int total_key_bits, int32_t *dir,
                                int32_t *counters, hipStream_t s) {
    const int db = neighbor_dir_bits(total_key_bits);
    const int64_t nb = (int64_t(1) << db) + 1;
    k_key_directory<<<grid_for(nb, 256), 256, 0, s>>>(leaf_key, L, db, total_key_bits - db, dir, counters);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

namespace {
NbrTree make_tree(const uint64_t *leaf_key, const int8_t *leaf_level, const int32_t *leaf_start, int64_t L,
                  int key_bits, int inst_shift, const int32_t *dir, int total_key_bits, const NbrTargets *tg) {
    NbrTree t;
    t.leaf_key = leaf_key;
    t.leaf_level = leaf_level;
    t.leaf_start = leaf_start;
    t.dir = dir;
    t.L = L;
    t.tkey = tg ? tg->leaf_key : leaf_key;
    t.tlevel = tg ? tg->leaf_level : leaf_level;
    t.Lt = tg ? tg->L : L;
    t.key_bits = key_bits;
    t.inst_shift = inst_shift;
    t.dir_bits = neighbor_dir_bits(total_key_bits);
    t.dir_shift = total_key_bits - t.dir_bits;
    return t;
}
}  // namespace

p2p_status launch_neighbors_count(const uint64_t *leaf_key, const int8_t *leaf_level, int64_t L,
                                  int key_bits, int inst_shift, const int32_t *dir, int total_key_bits,
                                  const int32_t *leaf_start, int32_t *counts, int32_t *segs,
                                  int32_t *slots, int8_t *slot_code, int32_t *counters, int32_t *heavy,
                                  hipStream_t s, const NbrTargets *tg) {
    const NbrTree t = make_tree(leaf_key, leaf_level, leaf_start, L, key_bits, inst_shift, dir, total_key_bits, tg);
    if (t.Lt <= 0) return P2P_OK;
#define P2P_NBR_COUNT(PER)                                                                             \
    k_neighbors<kNbrCount, PER><<<grid_for(t.Lt, kNbrWaves), 64 * kNbrWaves, 0, s>>>(                 \
        t, counts, segs, slots, slot_code, counters, heavy, nullptr, nullptr, nullptr);                 \
    P2P_LAUNCH_CHECK();                                                                                \
    k_neighbors_heavy<kNbrCount, PER><<<kHeavyGrid, 64 * kHeavyWaves, 0, s>>>(                        \
        t, counts, segs, slots, slot_code, counters, heavy, nullptr, nullptr, nullptr)
    if (slot_code) { P2P_NBR_COUNT(true); } else { P2P_NBR_COUNT(false); }
#undef P2P_NBR_COUNT
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_nbr_totals(const int64_t *start, const int64_t *seg_scan, const int32_t *counters,
                             int64_t L, int64_t *out, hipStream_t s) {
    k_nbr_totals<<<1, 1, 0, s>>>(start, seg_scan, counters, L, out);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_neighbors_fill(const uint64_t *leaf_key, const int8_t *leaf_level, int64_t L,
                                 int key_bits, int inst_shift, const int32_t *dir, int total_key_bits,
                                 const int32_t *counts, const int32_t *slots, const int8_t *slot_code,
                                 int32_t *counters, const int32_t *heavy, bool any_overflow,
                                 const int64_t *nbr_start, int32_t *nbr_idx, int8_t *nbr_shift, hipStream_t s,
                                 const NbrTargets *tg) {
    const NbrTree t = make_tree(leaf_key, leaf_level, nullptr, L, key_bits, inst_shift, dir, total_key_bits, tg);
    if (t.Lt <= 0) return P2P_OK;
    k_compact_slots<<<grid_for(t.Lt * kNbrSlots, 256), 256, 0, s>>>(counts, slots, slot_code, nbr_start, t.Lt,
                                                                    nbr_idx, nbr_shift);
    P2P_LAUNCH_CHECK();
    if (any_overflow) {
        int32_t *cn = const_cast<int32_t *>(counts);
#define P2P_NBR_FILL(PER)                                                                              \
        k_neighbors<kNbrFill, PER><<<grid_for(t.Lt, kNbrWaves), 64 * kNbrWaves, 0, s>>>(              \
            t, cn, nullptr, nullptr, nullptr, counters, nullptr, nbr_start, nbr_idx, nbr_shift);       \
        P2P_LAUNCH_CHECK();                                                                            \
        k_neighbors_heavy<kNbrFill, PER><<<kHeavyGrid, 64 * kHeavyWaves, 0, s>>>(                     \
            t, cn, nullptr, nullptr, nullptr, counters, heavy, nbr_start, nbr_idx, nbr_shift)
        if (slot_code) { P2P_NBR_FILL(true); } else { P2P_NBR_FILL(false); }
#undef P2P_NBR_FILL
        P2P_LAUNCH_CHECK();
    }
    return P2P_OK;
}

}  // namespace p2p
