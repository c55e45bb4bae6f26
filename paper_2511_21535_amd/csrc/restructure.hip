// Restructure to the redundant layout (Sec. 1.1, Sec. 5.2.1) and the gather-to-sorted-order
// permutations it and the gather layout share.
//
// The redundant segment of target leaf A is the concatenation, for B in
// nbr(A) in order, of B's sorted rows.  Rows are first moved from caller
// order into sorted order (one pass, N rows), then every segment is filled
// with coalesced copies, walking the segment in row order and locating the
// source leaf of each row in the prefix of neighbour occupancies kept in LDS.
#include <algorithm>

#include "p2p_internal.h"

namespace p2p {
namespace {

// Streaming stores for the redundant segments of a large layout: written once
// here and read once by the evaluation, so they are kept from displacing the
// sorted source rows (re-read by about 27 target leaves each) in L2.  A layout
// that fits the last-level cache is stored normally, where the evaluation
// finds it.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));
typedef uint32_t nt_u2 __attribute__((ext_vector_type(2)));

__device__ inline void stream_store(float4 *d, const float4 &v) {
    const nt_f4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f4 *>(d));
}
__device__ inline void stream_store(Row4d *d, const Row4d &v) {
    const nt_d2 a = {v.x, v.y}, b = {v.z, v.w};
    __builtin_nontemporal_store(a, reinterpret_cast<nt_d2 *>(d));
    __builtin_nontemporal_store(b, reinterpret_cast<nt_d2 *>(d) + 1);
}
__device__ inline void stream_store(uint4 *d, const uint4 &v) {
    const nt_u4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_u4 *>(d));
}
__device__ inline void stream_store(uint2 *d, const uint2 &v) {
    const nt_u2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_u2 *>(d));
}
__device__ inline void stream_store(uint32_t *d, const uint32_t &v) { __builtin_nontemporal_store(v, d); }

template <bool NT, class T>
__device__ inline void put_row(T *d, const T &v) {
    if constexpr (NT)
        stream_store(d, v);
    else
        *d = v;
}

// Segment length of every target leaf A (the points of the leaves in nbr(A))
// and the offset of A's own rows in it (the points of the entries listed
// before A's unshifted image, the lists being ascending in (image code, B)):
// 16 lanes per leaf, lanes across the list, two sums over the 16 lanes.
constexpr int kSegLanes = 16;

__global__ __launch_bounds__(256) void k_seg_lengths(const int32_t *__restrict__ leaf_start,
                                                     const int64_t *__restrict__ nbr_start,
                                                     const int32_t *__restrict__ nbr_idx,
                                                     const int8_t *__restrict__ nbr_shift, int64_t L,
                                                     int32_t *__restrict__ seg_len,
                                                     int32_t *__restrict__ red_self, int self_in_list) {
    const int sub = threadIdx.x % kSegLanes;
    const int64_t A = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kSegLanes;
    if (A >= L) return;     // whole 16-lane groups leave together
    int32_t len = 0, before = 0;
    for (int64_t e = nbr_start[A] + sub; e < nbr_start[A + 1]; e += kSegLanes) {
        const int32_t B = nbr_idx[e];
        const int code = nbr_shift ? nbr_shift[e] : 13;
        const int32_t occ = leaf_start[B + 1] - leaf_start[B];
        len += occ;
        if (code < 13 || (code == 13 && B < A)) before += occ;
    }
#pragma unroll
    for (int o = kSegLanes / 2; o > 0; o >>= 1) {
        len += __shfl_xor(len, o, kSegLanes);
        before += __shfl_xor(before, o, kSegLanes);
    }
    if (sub == 0) {
        seg_len[A] = len;
        red_self[A] = self_in_list ? before : -1;
    }
}

// Rows of upr units (a unit is the widest of 16, 8 or 4 bytes that divides the
// row): one thread per unit, UN units per thread in flight.
template <class U, int UN, class I>
__global__ __launch_bounds__(256) void k_permute_units(const U *__restrict__ src,
                                                       const int32_t *__restrict__ perm, I units,
                                                       I upr, U *__restrict__ dst) {
    const I base = static_cast<I>(blockIdx.x) * (256 * UN) + threadIdx.x;
    // units past the end repeat the last unit (same bytes, same place), so the
    // loads and stores carry no condition
    U v[UN];
#pragma unroll
    for (int k = 0; k < UN; ++k) {
        const I u = min(base + 256 * k, units - 1);
        const I s = u / upr;
        v[k] = src[static_cast<uint64_t>(perm[s]) * upr + (u - s * upr)];
    }
#pragma unroll
    for (int k = 0; k < UN; ++k) dst[min(base + 256 * k, units - 1)] = v[k];
}

// Four caller-order planes into sorted rows, in one pass: each thread reads
// one caller index from the four planes (coalesced) and writes its 32-byte row
// to the sorted slot iperm[i] (one aligned 32-byte write, where gathering
// would fetch a separate cache line from every plane).
__global__ void k_scatter4(const double *__restrict__ a, const double *__restrict__ b,
                           const double *__restrict__ c, const double *__restrict__ d,
                           const int32_t *__restrict__ iperm, int64_t n, Row4d *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[iperm[i]] = Row4d{a[i], b[i], c[i], d[i]};
}


constexpr int kCopyBlock = 256;
constexpr int kCopyNbrChunk = 256;   // near-list entries held in LDS at once

// Loads one chunk of A's near list into LDS: s_first[b] = first sorted slot of
// neighbour b, s_pre[b] = rows of the chunk before neighbour b, s_pre[nc] = rows
// in the chunk.  Called by the whole block.
__device__ int64_t load_nbr_chunk(const int32_t *__restrict__ leaf_start,
                                  const int32_t *__restrict__ nbr_idx, int64_t c0, int nc,
                                  int64_t *s_pre, int32_t *s_first, int64_t *s_w) {
    int32_t occ = 0, first = 0;
    if (static_cast<int>(threadIdx.x) < nc) {
        const int32_t B = nbr_idx[c0 + threadIdx.x];
        first = leaf_start[B];
        occ = leaf_start[B + 1] - first;
    }
    s_first[threadIdx.x] = first;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = occ;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int64_t woff = 0, tot = 0;
    for (int q = 0; q < kCopyBlock / 64; ++q) {
        if (q < w) woff += s_w[q];
        tot += s_w[q];
    }
    s_pre[threadIdx.x] = woff + x - occ;
    if (threadIdx.x == 0) s_pre[nc] = tot;
    __syncthreads();
    return tot;
}

// Gravity payload, one wavefront per target leaf (four per workgroup, no
// workgroup barriers).  Lanes load a chunk of 64 near-list entries and form
// the exclusive prefix of their occupancies with wave shuffles; each lane then
// marks the rows of its neighbour in an LDS map (row -> neighbour), and the
// segment is copied eight rows per lane at a time, every row finding its
// source through the map (or, for a chunk of more than kMapRows rows, by a
// forward walk over the prefix).  FP32_MIXED rows are written as float4
// (x - c_A, y - c_A, z - c_A, m) with c_A the centre of the target leaf, the
// difference taken in double.  PER (periodic lists): each row is first
// shifted by its entry's image, (x + s) in double.
constexpr int kMapRows = 4096;
constexpr int kRowsPerLane = 8;

// GATH (remote sources, a thin layer of another domain): rows read through the
// source tree's perm from the caller-order planes, instead of sorting all of
// that domain's points first.
template <bool MIXED, bool NT, bool PER, bool GATH>
__global__ __launch_bounds__(256) void k_copy_segments_grav(
    const Row4d *__restrict__ sorted, PermRows pr, const uint64_t *__restrict__ leaf_key,
    const int8_t *__restrict__ leaf_level, const int32_t *__restrict__ leaf_start,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int8_t *__restrict__ nbr_shift, const int64_t *__restrict__ red_start, int64_t L,
    Row4d *__restrict__ d8, float4 *__restrict__ d4) {
    __shared__ int32_t s_pre[4][65];
    __shared__ int32_t s_first[4][64];
    __shared__ int32_t s_code[PER ? 4 : 1][64];
    __shared__ uint8_t s_map[4][kMapRows];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t A = p2pd::xcd_contiguous(blockIdx.x, gridDim.x) * 4 + w;
    if (A >= L) return;
    double c[3] = {0.0, 0.0, 0.0};
    if (MIXED) {
        const uint64_t k = leaf_key[A];
        const double half = 0.5 * static_cast<double>(1u << (20 - leaf_level[A]));
        c[0] = (static_cast<double>(p2pd::compact3(k)) + half) * 0x1p-20;
        c[1] = (static_cast<double>(p2pd::compact3(k >> 1)) + half) * 0x1p-20;
        c[2] = (static_cast<double>(p2pd::compact3(k >> 2)) + half) * 0x1p-20;
    }
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
    int64_t out = red_start[A];
    for (int64_t c0 = e0; c0 < e1; c0 += 64) {
        const int nc = static_cast<int>(min<int64_t>(64, e1 - c0));
        int32_t occ = 0, first = 0, code = 13;
        if (lane < nc) {
            const int32_t B = nbr_idx[c0 + lane];
            first = leaf_start[B];
            occ = leaf_start[B + 1] - first;
            if constexpr (PER) code = nbr_shift[c0 + lane];
        }
        int32_t inc = occ;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        s_pre[w][lane] = inc - occ;
        s_first[w][lane] = first;
        if constexpr (PER) s_code[w][lane] = code;
        const int32_t rows = __shfl(inc, 63, 64);
        if (lane == 0) s_pre[w][64] = rows;
        const bool use_map = rows <= kMapRows;
        if (use_map)
            for (int32_t r = inc - occ; r < inc; ++r) s_map[w][r] = static_cast<uint8_t>(lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int b = 0;
        auto src_row = [&](int32_t p) {
            int bb;
            if (use_map) {
                bb = s_map[w][p];
            } else {
                while (b + 1 < nc && s_pre[w][b + 1] <= p) ++b;
                bb = b;
            }
            const int64_t slot = s_first[w][bb] + (p - s_pre[w][bb]);
            Row4d v;
            if constexpr (GATH) {
                const int64_t j = pr.perm[slot];
                v = Row4d{pr.x[j], pr.y[j], pr.z[j], pr.m[j]};
            } else {
                v = sorted[slot];
            }
            if constexpr (PER) {
                const int cd = s_code[w][bb];
                v.x += static_cast<double>(cd % 3 - 1);
                v.y += static_cast<double>((cd / 3) % 3 - 1);
                v.z += static_cast<double>(cd / 9 - 1);
            }
            return v;
        };
        // all loads of a group are issued before any of its stores; lanes
        // past the end take the last row again and store it to its own place
        // once more (the same bytes), so no load or store is conditional
        for (int32_t p0 = 0; p0 < rows; p0 += 64 * kRowsPerLane) {
            Row4d v[kRowsPerLane];
#pragma unroll
            for (int u = 0; u < kRowsPerLane; ++u) v[u] = src_row(min(p0 + 64 * u + lane, rows - 1));
#pragma unroll
            for (int u = 0; u < kRowsPerLane; ++u) {
                const int64_t d = out + min(p0 + 64 * u + lane, rows - 1);
                if constexpr (MIXED)
                    put_row<NT>(d4 + d, make_float4(static_cast<float>(v[u].x - c[0]),
                                                     static_cast<float>(v[u].y - c[1]),
                                                     static_cast<float>(v[u].z - c[2]),
                                                     static_cast<float>(v[u].w)));
                else
                    put_row<NT>(d8 + d, v[u]);
            }
        }
        out += rows;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Rows of upr units (Helmholtz right-hand sides): one workgroup per target
// leaf.  The rows of one neighbour are contiguous in sorted order, so a segment
// is a concatenation of runs; in unit space, unit u of the chunk belongs to
// the run b with s_pre[b] * upr <= u, and its source is u shifted by that
// run's (first - pre) * upr.  Threads take units tid, tid + 256, ...; each
// walks its run index forward (units only increase) and issues UN loads before
// its UN stores, none of them under a condition.
template <class U, int UN, bool NT>
__global__ __launch_bounds__(kCopyBlock) void k_copy_segments_units(
    const U *__restrict__ sorted, int64_t upr, const int32_t *__restrict__ leaf_start,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, int64_t L, U *__restrict__ dst, BoxSegments boxes) {
    __shared__ int64_t s_pre[kCopyNbrChunk + 1];
    __shared__ int32_t s_first[kCopyNbrChunk];
    __shared__ int64_t s_w[kCopyBlock / 64];
    const int64_t A = p2pd::xcd_contiguous(blockIdx.x, gridDim.x);
    if (A >= L) return;
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
    int64_t out;
    if (boxes.box_rows > 0) {
        // full boxes: the offsets follow from the list positions, no scan needed
        out = static_cast<int64_t>(boxes.box_rows) * e0;
        if (threadIdx.x == 0) {
            boxes.red_start[A] = out;
            if (A == L - 1) boxes.red_start[L] = static_cast<int64_t>(boxes.box_rows) * e1;
        }
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kCopyBlock)
            if (nbr_idx[e] == A) boxes.red_self[A] = boxes.box_rows * static_cast<int32_t>(e - e0);
    } else {
        out = red_start[A];
    }
    for (int64_t c0 = e0; c0 < e1; c0 += kCopyNbrChunk) {
        const int nc = static_cast<int>(min<int64_t>(kCopyNbrChunk, e1 - c0));
        const int64_t rows = load_nbr_chunk(leaf_start, nbr_idx, c0, nc, s_pre, s_first, s_w);
        const int64_t units = rows * upr;
        U *__restrict__ d = dst + out * upr;
        int b = 0;
        int64_t next = (nc > 1) ? s_pre[1] * upr : units;    // first unit of run b + 1
        int64_t shift = (static_cast<int64_t>(s_first[0]) - s_pre[0]) * upr;
        for (int64_t u0 = threadIdx.x; u0 < units; u0 += kCopyBlock * UN) {
            // units past the end repeat the last unit (same bytes, same place)
            U v[UN];
#pragma unroll
            for (int k = 0; k < UN; ++k) {
                const int64_t u = min(u0 + kCopyBlock * k, units - 1);
                while (u >= next) {
                    ++b;
                    next = (b + 1 < nc) ? s_pre[b + 1] * upr : units;
                    shift = (static_cast<int64_t>(s_first[b]) - s_pre[b]) * upr;
                }
                v[k] = sorted[u + shift];
            }
#pragma unroll
            for (int k = 0; k < UN; ++k) put_row<NT>(d + min(u0 + kCopyBlock * k, units - 1), v[k]);
        }
        out += rows;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- tiles --
// Block-level redundancy on grid trees (Sec. 3.5: for dense, regular
// distributions the data are duplicated per block of work, not per thread).
// A tile is the set of boxes of one instance whose box coordinates agree after
// division by the grain g (a power of two): an aligned g x g x g block, which
// in Morton order is one contiguous run of leaves, and whose first leaf is the
// block's lower corner.  The tile's segment holds the rows of the union of its
// boxes' near lists (its halo: the boxes of the window of (g+2)^3 box cells
// around it that exist), in ascending leaf id, every box 64 rows.
constexpr int kTileMaxGrain = 4;
constexpr int kTileWin = (kTileMaxGrain + 2) * (kTileMaxGrain + 2) * (kTileMaxGrain + 2);

__device__ inline void box_cell(uint64_t key, uint64_t local_mask, int c[3]) {
    const uint64_t l = key & local_mask;
    c[0] = static_cast<int>(p2pd::compact3(l)) >> 2;
    c[1] = static_cast<int>(p2pd::compact3(l >> 1)) >> 2;
    c[2] = static_cast<int>(p2pd::compact3(l >> 2)) >> 2;
}

// One 64-lane workgroup per leaf; only the first leaf of a tile works.  The
// halo is marked in a window of box cells (every entry of the tile's lists
// writes its source's id into its cell; entries naming one box write the same
// value), then each marked cell is ranked among the marked ones by id.
// FILL = false: cnt[A] = halo size at the tile's first leaf A, 0 elsewhere.
// FILL = true: with hs = the exclusive scan of cnt, the tile's halo ids go to
// halo_idx[hs[A] ..], every entry e of its lists gets red_row[e] = 64 (hs[A]
// + rank of its source), and every leaf of the tile red_start = 64 hs[A].
template <bool FILL>
__global__ __launch_bounds__(64) void k_tile_halo(const uint64_t *__restrict__ leaf_key,
                                                  const int64_t *__restrict__ nbr_start,
                                                  const int32_t *__restrict__ nbr_idx, int64_t L, int key_bits,
                                                  int lg, int64_t *__restrict__ cnt,
                                                  const int64_t *__restrict__ hs, int32_t *__restrict__ halo_idx,
                                                  int64_t *__restrict__ red_row, int64_t *__restrict__ red_start) {
    __shared__ int32_t s_id[kTileWin];
    __shared__ int32_t s_rank[kTileWin];
    const int64_t A = blockIdx.x;
    if (A >= L) return;
    const int lane = threadIdx.x;
    const int shift = 3 * (2 + lg);
    const uint64_t kA = leaf_key[A];
    const uint64_t tk = kA >> shift;
    const bool first = A == 0 || (leaf_key[A - 1] >> shift) != tk;
    if (!first) {
        if (!FILL && lane == 0) cnt[A] = 0;
        return;
    }
    const int g = 1 << lg, gw = g + 2, W = gw * gw * gw;
    // the tile's leaves: A .. A + nb - 1 (contiguous in key order, at most g^3 <= 64)
    const bool mine = lane < g * g * g && A + lane < L && (leaf_key[A + lane] >> shift) == tk;
    const int nb = __popcll(__ballot(mine));
    const uint64_t local_mask = (1ull << (3 * key_bits)) - 1ull;
    int o[3];
    box_cell(kA, local_mask, o);
    for (int c = lane; c < W; c += 64) s_id[c] = -1;
    __syncthreads();
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + nb];
    auto cell_of = [&](int32_t B) {
        int c[3];
        box_cell(leaf_key[B], local_mask, c);
        return (c[0] - o[0] + 1) + gw * ((c[1] - o[1] + 1) + gw * (c[2] - o[2] + 1));
    };
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int32_t B = nbr_idx[e];
        s_id[cell_of(B)] = B;
    }
    __syncthreads();
    int marked = 0;
    for (int c = lane; c < W; c += 64) {
        const int32_t id = s_id[c];
        int r = 0;
        if (id >= 0)
            for (int d = 0; d < W; ++d) {
                const int32_t v = s_id[d];
                r += (v >= 0 && v < id) ? 1 : 0;
            }
        s_rank[c] = r;
        marked += id >= 0 ? 1 : 0;
    }
    if constexpr (!FILL) {
        for (int off = 32; off > 0; off >>= 1) marked += __shfl_xor(marked, off, 64);
        if (lane == 0) cnt[A] = marked;
    } else {
        __syncthreads();
        const int64_t h0 = hs[A];
        for (int c = lane; c < W; c += 64)
            if (s_id[c] >= 0) halo_idx[h0 + s_rank[c]] = s_id[c];
        for (int64_t e = e0 + lane; e < e1; e += 64) red_row[e] = 64 * (h0 + s_rank[cell_of(nbr_idx[e])]);
        if (lane < nb) red_start[A + lane] = 64 * h0;
        if (lane == 0 && A + nb == L) red_start[L] = 64 * hs[L];
    }
}

// The tile segments' rows: box halo_idx[j] goes to rows [64 j, 64 j + 64),
// read from caller order through perm (a grid box's rows are runs of 4
// consecutive caller rows, whole rows of upr units each).  Workgroups stride
// over the halo boxes; each thread keeps UN units in flight.
template <class U, int UN, bool NT>
__global__ __launch_bounds__(kCopyBlock) void k_tile_copy(const U *__restrict__ q, int64_t upr, int lg_upr,
                                                         const int32_t *__restrict__ leaf_start,
                                                         const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ halo_idx, int64_t H,
                                                         U *__restrict__ dst) {
    const int64_t units = 64 * upr;
    for (int64_t j = blockIdx.x; j < H; j += gridDim.x) {
        const int32_t r0 = leaf_start[halo_idx[j]];
        U *__restrict__ d = dst + j * units;
        for (int64_t u0 = threadIdx.x; u0 < units; u0 += kCopyBlock * UN) {
            U v[UN];
#pragma unroll
            for (int k = 0; k < UN; ++k) {
                // units past the end repeat the last unit (same bytes, same place)
                const int64_t u = min(u0 + kCopyBlock * k, units - 1);
                const int64_t row = lg_upr >= 0 ? (u >> lg_upr) : u / upr;
                v[k] = q[static_cast<int64_t>(perm[r0 + row]) * upr + (u - row * upr)];
            }
#pragma unroll
            for (int k = 0; k < UN; ++k) put_row<NT>(d + min(u0 + kCopyBlock * k, units - 1), v[k]);
        }
    }
}

template <class U>
p2p_status tile_copy_units(const void *q, int64_t row_bytes, const int32_t *leaf_start, const int32_t *perm,
                           const int32_t *halo_idx, int64_t H, void *dst, bool streaming, hipStream_t s) {
    const int64_t upr = row_bytes / static_cast<int64_t>(sizeof(U));
    int lg = -1;
    for (int b = 0; b < 40; ++b)
        if ((int64_t(1) << b) == upr) lg = b;
    int dev = 0, cus = 0;
    P2P_HIP(hipGetDevice(&dev));
    P2P_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(H, static_cast<int64_t>(cus) * 8));
    if (streaming)
        k_tile_copy<U, 4, true><<<grid, kCopyBlock, 0, s>>>(static_cast<const U *>(q), upr, lg, leaf_start, perm,
                                                            halo_idx, H, static_cast<U *>(dst));
    else
        k_tile_copy<U, 4, false><<<grid, kCopyBlock, 0, s>>>(static_cast<const U *>(q), upr, lg, leaf_start, perm,
                                                             halo_idx, H, static_cast<U *>(dst));
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace

p2p_status launch_seg_lengths(const int32_t *leaf_start, const int64_t *nbr_start,
                              const int32_t *nbr_idx, const int8_t *nbr_shift, int64_t L,
                              int32_t *seg_len, int32_t *red_self, bool self_in_list, hipStream_t s) {
    if (L <= 0) return P2P_OK;
    k_seg_lengths<<<grid_for(L * kSegLanes, 256), 256, 0, s>>>(leaf_start, nbr_start, nbr_idx, nbr_shift, L,
                                                                seg_len, red_self, self_in_list ? 1 : 0);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

namespace {

// Widest unit (16, 8 or 4 bytes) that divides a row of `row_bytes`.
int unit_bytes(int64_t row_bytes) {
    return (row_bytes % 16 == 0) ? 16 : (row_bytes % 8 == 0) ? 8 : 4;
}

template <class U>
p2p_status permute_units(const void *src, const int32_t *perm, int64_t n, int64_t row_bytes,
                         void *dst, hipStream_t s) {
    constexpr int UN = 4;
    const uint64_t upr = static_cast<uint64_t>(row_bytes) / sizeof(U);
    const uint64_t units = static_cast<uint64_t>(n) * upr;
    const uint64_t blocks = (units + 256 * UN - 1) / (256 * UN);
    // 32-bit unit indices while they fit (with room for the last block's overshoot)
    if (units + 256 * UN < (uint64_t(1) << 32))
        k_permute_units<U, UN, uint32_t><<<static_cast<unsigned>(blocks), 256, 0, s>>>(
            static_cast<const U *>(src), perm, static_cast<uint32_t>(units),
            static_cast<uint32_t>(upr), static_cast<U *>(dst));
    else
        k_permute_units<U, UN, uint64_t><<<static_cast<unsigned>(blocks), 256, 0, s>>>(
            static_cast<const U *>(src), perm, units, upr, static_cast<U *>(dst));
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

// Box-grain segments of full grid boxes (64 rows each) with 8- or 16-byte
// rows: near-list entry e copies its source box's 64 rows, 2^LGU 16-byte
// units, to units [e 2^LGU, (e + 1) 2^LGU) of the layout, one unit per thread,
// so that each group of 2^LGU lanes moves one contiguous run.  Threads below L
// also write box A's segment offset and the position of its own rows.
template <int LGU, bool NT>
__global__ __launch_bounds__(256) void k_copy_box_entries(const uint4 *__restrict__ sorted,
                                                          const int32_t *__restrict__ leaf_start,
                                                          const int64_t *__restrict__ nbr_start,
                                                          const int32_t *__restrict__ nbr_idx, int64_t L,
                                                          uint4 *__restrict__ dst, BoxSegments boxes) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t < L) {
        const int64_t e0 = nbr_start[t], e1 = nbr_start[t + 1];
        boxes.red_start[t] = static_cast<int64_t>(boxes.box_rows) * e0;
        if (t == L - 1) boxes.red_start[L] = static_cast<int64_t>(boxes.box_rows) * e1;
        for (int64_t e = e0; e < e1; ++e)
            if (nbr_idx[e] == t) boxes.red_self[t] = boxes.box_rows * static_cast<int32_t>(e - e0);
    }
    if (t >= (boxes.entries << LGU)) return;
    const int64_t e = t >> LGU;
    const int k = static_cast<int>(t & ((1 << LGU) - 1));
    // 64 rows are 2^LGU units, so row r starts at unit r 2^LGU / 64 (r a multiple of 64)
    const int64_t src = (static_cast<int64_t>(leaf_start[nbr_idx[e]]) << LGU) >> 6;
    put_row<NT>(dst + t, sorted[src + k]);
}

template <class U>
p2p_status copy_units(const void *sorted, int64_t row_bytes, const int32_t *leaf_start,
                      const int64_t *nbr_start, const int32_t *nbr_idx, const int64_t *red_start,
                      int64_t L, void *dst, bool streaming, hipStream_t s, BoxSegments boxes) {
    const int64_t upr = row_bytes / static_cast<int64_t>(sizeof(U));
    if (streaming)
        k_copy_segments_units<U, 4, true><<<static_cast<unsigned>(L), kCopyBlock, 0, s>>>(
            static_cast<const U *>(sorted), upr, leaf_start, nbr_start, nbr_idx, red_start, L,
            static_cast<U *>(dst), boxes);
    else
        k_copy_segments_units<U, 4, false><<<static_cast<unsigned>(L), kCopyBlock, 0, s>>>(
            static_cast<const U *>(sorted), upr, leaf_start, nbr_start, nbr_idx, red_start, L,
            static_cast<U *>(dst), boxes);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace

template <class T>
p2p_status launch_permute_rows(const T *src, const int32_t *perm, int64_t n, int64_t row_len,
                               T *dst, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    if (!src || !perm || !dst) return fail(P2P_EINVAL, "internal: row permutation with a null array");
    const int64_t rb = row_len * static_cast<int64_t>(sizeof(T));
    switch (unit_bytes(rb)) {
    case 16: return permute_units<uint4>(src, perm, n, rb, dst, s);
    case 8: return permute_units<uint2>(src, perm, n, rb, dst, s);
    default: return permute_units<uint32_t>(src, perm, n, rb, dst, s);
    }
}

p2p_status launch_scatter4(const double *a, const double *b, const double *c, const double *d,
                           const int32_t *iperm, int64_t n, Row4d *out, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    if (!a || !b || !c || !d || !iperm || !out) return fail(P2P_EINVAL, "internal: row scatter with a null array");
    k_scatter4<<<grid_for(n, 256), 256, 0, s>>>(a, b, c, d, iperm, n, out);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_copy_segments_gravity(const Row4d *sorted, const uint64_t *leaf_key,
                                        const int8_t *leaf_level, const int32_t *leaf_start,
                                        const int64_t *nbr_start, const int32_t *nbr_idx,
                                        const int8_t *nbr_shift, const int64_t *red_start, int64_t L,
                                        Row4d *d8, float4 *d4, bool streaming, hipStream_t s,
                                        const PermRows *pr) {
    if (L <= 0) return P2P_OK;
    const unsigned g = grid_for(L, 4);
    const PermRows prv = pr ? *pr : PermRows{};
#define P2P_COPY_GRAV(M, NT, PER, G)                                                                      \
    k_copy_segments_grav<M, NT, PER, G><<<g, 256, 0, s>>>(sorted, prv, leaf_key, leaf_level, leaf_start, \
                                                          nbr_start, nbr_idx, nbr_shift, red_start, L, d8, d4)
#define P2P_COPY_GRAV_NT(M, PER, G) \
    if (streaming) P2P_COPY_GRAV(M, true, PER, G); else P2P_COPY_GRAV(M, false, PER, G)
#define P2P_COPY_GRAV_G(M, PER) \
    if (pr) { P2P_COPY_GRAV_NT(M, PER, true); } else { P2P_COPY_GRAV_NT(M, PER, false); }
    if (nbr_shift) {
        if (d4) { P2P_COPY_GRAV_G(true, true) } else { P2P_COPY_GRAV_G(false, true) }
    } else {
        if (d4) { P2P_COPY_GRAV_G(true, false) } else { P2P_COPY_GRAV_G(false, false) }
    }
#undef P2P_COPY_GRAV_G
#undef P2P_COPY_GRAV_NT
#undef P2P_COPY_GRAV
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

template <class T>
p2p_status launch_copy_segments(const T *sorted, int64_t row_len, const int32_t *leaf_start,
                                const int64_t *nbr_start, const int32_t *nbr_idx,
                                const int64_t *red_start, int64_t L, T *dst, bool streaming,
                                hipStream_t s, BoxSegments boxes) {
    if (L <= 0) return P2P_OK;
    if (boxes.box_rows > 0 && (!boxes.red_start || !boxes.red_self))
        return fail(P2P_EINVAL, "internal: box segments without their arrays");
    const int64_t rb = row_len * static_cast<int64_t>(sizeof(T));
    if (boxes.box_rows == 64 && (rb == 8 || rb == 16) && (reinterpret_cast<uintptr_t>(dst) & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(sorted) & 15) == 0) {
        // full grid boxes with one right-hand side (16-byte aligned layout): one
        // 16-byte unit per thread
        const int lgu = rb == 8 ? 5 : 6;
        const int64_t threads = std::max<int64_t>(L, boxes.entries << lgu);
        const unsigned grid = static_cast<unsigned>((threads + 255) / 256);
        const uint4 *src4 = reinterpret_cast<const uint4 *>(sorted);
        uint4 *dst4 = reinterpret_cast<uint4 *>(dst);
#define P2P_CBE(G, N) \
    k_copy_box_entries<G, N><<<grid, 256, 0, s>>>(src4, leaf_start, nbr_start, nbr_idx, L, dst4, boxes)
        if (lgu == 5) { if (streaming) P2P_CBE(5, true); else P2P_CBE(5, false); }
        else { if (streaming) P2P_CBE(6, true); else P2P_CBE(6, false); }
#undef P2P_CBE
        P2P_LAUNCH_CHECK();
        return P2P_OK;
    }
    switch (unit_bytes(rb)) {
    case 16:
        return copy_units<uint4>(sorted, rb, leaf_start, nbr_start, nbr_idx, red_start, L, dst, streaming, s,
                                 boxes);
    case 8:
        return copy_units<uint2>(sorted, rb, leaf_start, nbr_start, nbr_idx, red_start, L, dst, streaming, s,
                                 boxes);
    default:
        return copy_units<uint32_t>(sorted, rb, leaf_start, nbr_start, nbr_idx, red_start, L, dst, streaming,
                                    s, boxes);
    }
}

p2p_status launch_tile_halo(const uint64_t *leaf_key, const int64_t *nbr_start, const int32_t *nbr_idx,
                            int64_t L, int key_bits, int grain, int64_t *cnt, const int64_t *hs,
                            int32_t *halo_idx, int64_t *red_row, int64_t *red_start, hipStream_t s) {
    if (L <= 0) return P2P_OK;
    int lg = 0;
    while ((1 << lg) < grain) ++lg;
    if ((1 << lg) != grain || grain > kTileMaxGrain) return fail(P2P_EINVAL, "internal: tile grain");
    if (!hs)
        k_tile_halo<false><<<static_cast<unsigned>(L), 64, 0, s>>>(leaf_key, nbr_start, nbr_idx, L, key_bits, lg,
                                                                   cnt, nullptr, nullptr, nullptr, nullptr);
    else
        k_tile_halo<true><<<static_cast<unsigned>(L), 64, 0, s>>>(leaf_key, nbr_start, nbr_idx, L, key_bits, lg,
                                                                  nullptr, hs, halo_idx, red_row, red_start);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_tile_copy(const void *q, int64_t row_bytes, const int32_t *leaf_start, const int32_t *perm,
                            const int32_t *halo_idx, int64_t H, void *dst, bool streaming, hipStream_t s) {
    if (H <= 0) return P2P_OK;
    switch (unit_bytes(row_bytes)) {
    case 16: return tile_copy_units<uint4>(q, row_bytes, leaf_start, perm, halo_idx, H, dst, streaming, s);
    case 8: return tile_copy_units<uint2>(q, row_bytes, leaf_start, perm, halo_idx, H, dst, streaming, s);
    default: return tile_copy_units<uint32_t>(q, row_bytes, leaf_start, perm, halo_idx, H, dst, streaming, s);
    }
}

template p2p_status launch_permute_rows<double>(const double *, const int32_t *, int64_t, int64_t,
                                                double *, hipStream_t);
template p2p_status launch_permute_rows<float2>(const float2 *, const int32_t *, int64_t, int64_t,
                                                float2 *, hipStream_t);
template p2p_status launch_permute_rows<double2>(const double2 *, const int32_t *, int64_t, int64_t,
                                                 double2 *, hipStream_t);
template p2p_status launch_copy_segments<double>(const double *, int64_t, const int32_t *,
                                                 const int64_t *, const int32_t *, const int64_t *,
                                                 int64_t, double *, bool, hipStream_t, BoxSegments);
template p2p_status launch_copy_segments<float>(const float *, int64_t, const int32_t *,
                                                const int64_t *, const int32_t *, const int64_t *,
                                                int64_t, float *, bool, hipStream_t, BoxSegments);
template p2p_status launch_copy_segments<float2>(const float2 *, int64_t, const int32_t *,
                                                 const int64_t *, const int32_t *, const int64_t *,
                                                 int64_t, float2 *, bool, hipStream_t, BoxSegments);
template p2p_status launch_copy_segments<double2>(const double2 *, int64_t, const int32_t *,
                                                  const int64_t *, const int32_t *, const int64_t *,
                                                  int64_t, double2 *, bool, hipStream_t, BoxSegments);

}  // namespace p2p
