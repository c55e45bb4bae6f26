// Restructure to the redundant layout (a3) and the gather-to-sorted-order
// permutations it and the gather layout share.
//
// The redundant segment of target leaf A is the concatenation, for B in
// nbr(A) in order, of B's sorted rows.  Rows are first permuted from caller
// order into sorted order (one pass, N rows), then every segment is filled
// with coalesced copies: a workgroup owns one target leaf and walks its
// segment in row order, locating the source leaf of each row by a binary
// search over the prefix of neighbour occupancies kept in LDS.
#include "p2p_internal.h"

namespace p2p {
namespace {

__global__ void k_seg_lengths(const int32_t *__restrict__ leaf_start,
                              const int64_t *__restrict__ nbr_start,
                              const int32_t *__restrict__ nbr_idx, int64_t L,
                              int64_t *__restrict__ seg_len, int32_t *__restrict__ red_self) {
    int64_t A = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (A >= L) return;
    int64_t len = 0, self = 0;
    for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
        const int32_t B = nbr_idx[e];
        if (B == A) self = len;
        len += leaf_start[B + 1] - leaf_start[B];
    }
    seg_len[A] = len;
    red_self[A] = static_cast<int32_t>(self);
}

// Rows of row_len elements: row_len == 1 one row per thread, otherwise one
// wave per row with lanes across it.
template <class T>
__global__ void k_permute_rows(const T *__restrict__ src, const int32_t *__restrict__ perm,
                               int64_t n, int row_len, T *__restrict__ dst) {
    if (row_len == 1) {
        const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
        if (s < n) dst[s] = src[perm[s]];
        return;
    }
    const int lane = threadIdx.x & 63;
    const int64_t s = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (s >= n) return;
    const int64_t from = static_cast<int64_t>(perm[s]) * row_len, to = s * row_len;
    for (int r = lane; r < row_len; r += 64) dst[to + r] = src[from + r];
}

// Four caller-order planes into sorted rows, in one pass.
__global__ void k_permute4(const double *__restrict__ a, const double *__restrict__ b,
                           const double *__restrict__ c, const double *__restrict__ d,
                           const int32_t *__restrict__ perm, int64_t n, Row4d *__restrict__ out) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    out[s] = Row4d{a[i], b[i], c[i], d[i]};
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
    if (threadIdx.x < nc) {
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

// Index of the last neighbour b < nc with s_pre[b] <= p.
__device__ inline int find_nbr(const int64_t *s_pre, int nc, int64_t p) {
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Gravity payload, one wavefront per target leaf (four per workgroup, no
// workgroup barriers).  Lanes load a chunk of 64 near-list entries, form the
// exclusive prefix of their occupancies with wave shuffles, and then copy the
// segment row by row; a row finds its source leaf by binary search over the
// prefix.  FP32_MIXED rows are written as float4 (x - c_A, y - c_A, z - c_A,
// m) with c_A the centre of the target leaf, the difference taken in double.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_copy_segments_grav(
    const Row4d *__restrict__ sorted, const uint64_t *__restrict__ leaf_key,
    const int8_t *__restrict__ leaf_level, const int32_t *__restrict__ leaf_start,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, int64_t L, Row4d *__restrict__ d8,
    float4 *__restrict__ d4) {
    __shared__ int32_t s_pre[4][65];
    __shared__ int32_t s_first[4][64];
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
        int32_t occ = 0, first = 0;
        if (lane < nc) {
            const int32_t B = nbr_idx[c0 + lane];
            first = leaf_start[B];
            occ = leaf_start[B + 1] - first;
        }
        int32_t inc = occ;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        s_pre[w][lane] = inc - occ;
        s_first[w][lane] = first;
        const int32_t rows = __shfl(inc, 63, 64);
        if (lane == 0) s_pre[w][64] = rows;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // rows p = lane + 64 j; the neighbour of each row is found by walking
        // forward from the previous row's (rows only increase), and the loads
        // of four rows are issued before any of them is used
        int b = 0;
        auto src_row = [&](int32_t p) {
            while (b + 1 < nc && s_pre[w][b + 1] <= p) ++b;
            return sorted[s_first[w][b] + (p - s_pre[w][b])];
        };
        auto put = [&](int64_t d, const Row4d &v) {
            if constexpr (MIXED)
                d4[d] = make_float4(static_cast<float>(v.x - c[0]), static_cast<float>(v.y - c[1]),
                                    static_cast<float>(v.z - c[2]), static_cast<float>(v.w));
            else
                d8[d] = v;
        };
        // full groups of 256 rows with no per-row condition, so the four loads
        // and the four stores of a group are all in flight together
        int32_t p0 = 0;
        for (; p0 + 256 <= rows; p0 += 256) {
            Row4d v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = src_row(p0 + 64 * u + lane);
#pragma unroll
            for (int u = 0; u < 4; ++u) put(out + p0 + 64 * u + lane, v[u]);
        }
        for (int32_t p = p0 + lane; p < rows; p += 64) put(out + p, src_row(p));
        out += rows;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Rows of row_len elements (Helmholtz right-hand sides): one wave per row,
// lanes across the row.
template <class T>
__global__ __launch_bounds__(kCopyBlock) void k_copy_segments_rows(
    const T *__restrict__ sorted, int row_len, const int32_t *__restrict__ leaf_start,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, T *__restrict__ dst) {
    __shared__ int64_t s_pre[kCopyNbrChunk + 1];
    __shared__ int32_t s_first[kCopyNbrChunk];
    __shared__ int64_t s_w[kCopyBlock / 64];
    const int64_t A = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
    int64_t out = red_start[A];
    for (int64_t c0 = e0; c0 < e1; c0 += kCopyNbrChunk) {
        const int nc = static_cast<int>(min<int64_t>(kCopyNbrChunk, e1 - c0));
        const int64_t rows = load_nbr_chunk(leaf_start, nbr_idx, c0, nc, s_pre, s_first, s_w);
        if (row_len == 1) {
            for (int64_t p = threadIdx.x; p < rows; p += kCopyBlock) {
                const int b = find_nbr(s_pre, nc, p);
                dst[out + p] = sorted[s_first[b] + (p - s_pre[b])];
            }
        } else {
            for (int64_t p = w; p < rows; p += kCopyBlock / 64) {
                const int b = find_nbr(s_pre, nc, p);
                const int64_t src = (s_first[b] + (p - s_pre[b])) * static_cast<int64_t>(row_len);
                const int64_t d = (out + p) * static_cast<int64_t>(row_len);
                for (int r = lane; r < row_len; r += 64) dst[d + r] = sorted[src + r];
            }
        }
        out += rows;
        __syncthreads();
    }
}

}  // namespace

p2p_status launch_seg_lengths(const int32_t *leaf_start, const int64_t *nbr_start,
                              const int32_t *nbr_idx, int64_t L, int64_t *seg_len,
                              int32_t *red_self, hipStream_t s) {
    if (L <= 0) return P2P_OK;
    k_seg_lengths<<<grid_for(L, 256), 256, 0, s>>>(leaf_start, nbr_start, nbr_idx, L, seg_len,
                                                  red_self);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

template <class T>
p2p_status launch_permute_rows(const T *src, const int32_t *perm, int64_t n, int64_t row_len,
                               T *dst, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    const int64_t threads = (row_len == 1) ? n : n * 64;
    k_permute_rows<T><<<grid_for(threads, 256), 256, 0, s>>>(src, perm, n,
                                                            static_cast<int>(row_len), dst);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_permute4(const double *a, const double *b, const double *c, const double *d,
                           const int32_t *perm, int64_t n, Row4d *out, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    k_permute4<<<grid_for(n, 256), 256, 0, s>>>(a, b, c, d, perm, n, out);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_copy_segments_gravity(const Row4d *sorted, const uint64_t *leaf_key,
                                        const int8_t *leaf_level, const int32_t *leaf_start,
                                        const int64_t *nbr_start, const int32_t *nbr_idx,
                                        const int64_t *red_start, int64_t L, Row4d *d8,
                                        float4 *d4, hipStream_t s) {
    if (L <= 0) return P2P_OK;
    const unsigned g = grid_for(L, 4);
    if (d4)
        k_copy_segments_grav<true><<<g, 256, 0, s>>>(sorted, leaf_key, leaf_level, leaf_start, nbr_start,
                                                     nbr_idx, red_start, L, d8, d4);
    else
        k_copy_segments_grav<false><<<g, 256, 0, s>>>(sorted, leaf_key, leaf_level, leaf_start, nbr_start,
                                                      nbr_idx, red_start, L, d8, d4);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

template <class T>
p2p_status launch_copy_segments(const T *sorted, int64_t row_len, const int32_t *leaf_start,
                                const int64_t *nbr_start, const int32_t *nbr_idx,
                                const int64_t *red_start, int64_t L, T *dst, hipStream_t s) {
    if (L <= 0) return P2P_OK;
    k_copy_segments_rows<T><<<static_cast<unsigned>(L), kCopyBlock, 0, s>>>(
        sorted, static_cast<int>(row_len), leaf_start, nbr_start, nbr_idx, red_start, dst);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

template p2p_status launch_permute_rows<double>(const double *, const int32_t *, int64_t, int64_t,
                                                double *, hipStream_t);
template p2p_status launch_permute_rows<float2>(const float2 *, const int32_t *, int64_t, int64_t,
                                                float2 *, hipStream_t);
template p2p_status launch_permute_rows<double2>(const double2 *, const int32_t *, int64_t, int64_t,
                                                 double2 *, hipStream_t);
template p2p_status launch_copy_segments<double>(const double *, int64_t, const int32_t *,
                                                 const int64_t *, const int32_t *, const int64_t *,
                                                 int64_t, double *, hipStream_t);
template p2p_status launch_copy_segments<float>(const float *, int64_t, const int32_t *,
                                                const int64_t *, const int32_t *, const int64_t *,
                                                int64_t, float *, hipStream_t);
template p2p_status launch_copy_segments<float2>(const float2 *, int64_t, const int32_t *,
                                                 const int64_t *, const int32_t *, const int64_t *,
                                                 int64_t, float2 *, hipStream_t);
template p2p_status launch_copy_segments<double2>(const double2 *, int64_t, const int32_t *,
                                                  const int64_t *, const int32_t *, const int64_t *,
                                                  int64_t, double2 *, hipStream_t);

}  // namespace p2p
