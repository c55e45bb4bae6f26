// Tree binning (Sec. 4: the stellar-dynamics tree is rebuilt every step):
// integer keys, and leaf boundaries over the sorted keys.
//
// Particles: c_d = floor(x_d 2^20), key = Morton(c).  The sort itself is
// radix_sort_pairs.  Leaves of an adaptive tree are found without walking
// the tree: over the sorted keys, let c[i] be the number of leading octal
// digits shared by keys i and i+1.  The node at level l that holds particle i
// contains exactly the run of neighbours reachable through pairs with
// c >= l, so its count is 1 + (run to the left) + (run to the right).  A
// particle's leaf is the shallowest node on its root path holding at most
// leaf_cap points (the split rule: split iff count > cap and level < depth),
// and that level is one more than the cap-th largest value of the merged,
// non-increasing sequences of running minima of c to the left and to the
// right of i.  A merge of leaf_cap steps finds it.
#include "p2p_internal.h"

namespace p2p {
namespace {

__global__ void k_particle_keys(const double *__restrict__ x, const double *__restrict__ y,
                                const double *__restrict__ z, int64_t n,
                                uint64_t *__restrict__ keys, int32_t *__restrict__ vals,
                                int32_t *__restrict__ bad) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {x[i], y[i], z[i]};
    uint32_t c[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ok = ok && (p[d] >= 0.0 && p[d] < 1.0);
        // x * 2^20 is exact; truncation of a non-negative value is floor
        c[d] = ok ? static_cast<uint32_t>(p[d] * 1048576.0) : 0u;
    }
    if (!ok) atomicOr(bad, 1);
    keys[i] = p2pd::morton3(c[0], c[1], c[2]);
    vals[i] = static_cast<int32_t>(i);
}

__global__ void k_grid_keys(const int32_t *__restrict__ n_side, const int64_t *__restrict__ off,
                            int32_t n_grids, int bits, int64_t n, uint64_t *__restrict__ keys,
                            int32_t *__restrict__ vals) {
    int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    // binary search of the instance: last g with off[g] <= p
    int lo = 0, hi = n_grids - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const int64_t ns = n_side[lo], loc = p - off[lo];
    const uint32_t i = static_cast<uint32_t>(loc % ns), j = static_cast<uint32_t>((loc / ns) % ns),
                   k = static_cast<uint32_t>(loc / (ns * ns));
    keys[p] = (static_cast<uint64_t>(lo) << (3 * bits)) | p2pd::morton3(i, j, k);
    vals[p] = static_cast<int32_t>(p);
}

// Leading octal digits shared by two depth-20 keys (60-bit keys in 64-bit words).
__device__ inline int common_digits(uint64_t a, uint64_t b) {
    uint64_t x = a ^ b;
    return x == 0 ? 20 : (__clzll(static_cast<long long>(x)) - 4) / 3;
}

__global__ void k_pair_common(const uint64_t *__restrict__ sk, int64_t n, uint8_t *__restrict__ c) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i + 1 < n) c[i] = static_cast<uint8_t>(common_digits(sk[i], sk[i + 1]));
}

// kind 0, leaf_cap > 0: adaptive level; kind 0, leaf_cap == 0: uniform depth.
__global__ void k_leaf_level_particles(const uint8_t *__restrict__ c, int64_t n, int depth,
                                       int leaf_cap, int8_t *__restrict__ level,
                                       int32_t *__restrict__ flag) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int l;
    if (leaf_cap == 0) {
        l = depth;
    } else {
        // merge the running minima to the left (pairs i-1, i-2, ...) and to the
        // right (pairs i, i+1, ...); -1 marks an exhausted side
        int64_t left = i - 1, right = i;
        int mL = 127, mR = 127;
        int cl = (left >= 0) ? static_cast<int>(c[left]) : -1;
        int cr = (right < n - 1) ? static_cast<int>(c[right]) : -1;
        int v = -1;
        for (int t = 0; t < leaf_cap; ++t) {
            int candL = (left >= 0) ? min(mL, cl) : -1;
            int candR = (right < n - 1) ? min(mR, cr) : -1;
            if (candL < 0 && candR < 0) { v = -1; break; }
            if (candL >= candR) {
                v = candL; mL = candL; --left;
                cl = (left >= 0) ? static_cast<int>(c[left]) : -1;
            } else {
                v = candR; mR = candR; ++right;
                cr = (right < n - 1) ? static_cast<int>(c[right]) : -1;
            }
        }
        l = min(depth, v + 1);
    }
    level[i] = static_cast<int8_t>(l);
    // a new leaf starts at i unless slot i-1 shares i's level-l node
    flag[i] = (i == 0 || static_cast<int>(c[i - 1]) < l) ? 1 : 0;
}

// The same leaf levels for leaf_cap <= 64 without the merge: slot i's leaf
// level is the coarsest level l whose node around i holds at most leaf_cap
// slots (the merge's last common-digit count v satisfies v + 1 = that level;
// past the node the merge only meets smaller counts), capped at depth.  The
// node at level l spans the run of counts >= l on either side of i, and no
// run longer than 64 matters, so a wave of 64 slots reads the counts of
// slots -64..127 around it as three ballots per level, and each lane measures
// its run with one leading- and one trailing-ones count.  Levels are tried
// from the root down until every lane has its answer.
__global__ __launch_bounds__(256) void k_leaf_level_ballot(const uint64_t *__restrict__ sk, int64_t n, int depth,
                                                           int leaf_cap, int8_t *__restrict__ level,
                                                           int32_t *__restrict__ flag) {
    __shared__ int8_t cs[256 + 128];   // cs[k] = c[b - 64 + k], -1 past either end
    const int64_t b = static_cast<int64_t>(blockIdx.x) * 256;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int k = t; k < 256 + 128; k += 256) {
        const int64_t j = b - 64 + k;
        cs[k] = (j >= 0 && j + 1 < n) ? static_cast<int8_t>(common_digits(sk[j], sk[j + 1])) : int8_t(-1);
    }
    __syncthreads();
    // this wave's window: c of slots (wave's first) - 64 + k, k < 192, in three registers
    const int c0 = cs[64 * wv + lane], c1 = cs[64 * wv + 64 + lane], c2 = cs[64 * wv + 128 + lane];
    const int sh = lane;   // the lane's own count c[i] sits at window bit 64 + lane
    int lev = -1;
    for (int l = 0; l <= 21; ++l) {
        const uint64_t W0 = __ballot(c0 >= l), W1 = __ballot(c1 >= l), W2 = __ballot(c2 >= l);
        // right: window bits 64 + lane .. 127 + lane; left: bits lane .. 63 + lane (top bit: c[i - 1])
        const uint64_t R = sh == 0 ? W1 : (W1 >> sh) | (W2 << (64 - sh));
        const uint64_t Lw = sh == 0 ? W0 : (W0 >> sh) | (W1 << (64 - sh));
        const int right = R == ~0ull ? 64 : __builtin_ctzll(~R);
        const int left = Lw == ~0ull ? 64 : __builtin_clzll(~Lw);
        if (lev < 0 && left + right + 1 <= leaf_cap) lev = l;
        if (__ballot(lev < 0) == 0) break;
    }
    const int64_t i = b + 64 * wv + lane;
    if (i >= n) return;
    const int l = min(depth, lev);
    level[i] = static_cast<int8_t>(l);
    flag[i] = (i == 0 || static_cast<int>(cs[64 * wv + 63 + lane]) < l) ? 1 : 0;
}

// The same leaf levels for leaf_cap <= kTileCap, a block of 256 slots at a
// time: the block first forms the common-digit counts of its slots and of
// leaf_cap slots on either side (the farthest the merge can reach) from the
// sorted keys into LDS, -1 past either end of the sequence, so the merge loop
// reads LDS instead of issuing a scattered byte load per step.
constexpr int kTileCap = 2048;
constexpr int kTileSlots = 256;
__global__ __launch_bounds__(kTileSlots) void k_leaf_level_tile(const uint64_t *__restrict__ sk, int64_t n,
                                                                  int depth, int leaf_cap,
                                                                  int8_t *__restrict__ level,
                                                                  int32_t *__restrict__ flag) {
    extern __shared__ int8_t cs[];   // cs[k] = c[b - leaf_cap + k], k < kTileSlots + 2 leaf_cap
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kTileSlots;
    const int t = threadIdx.x, w = kTileSlots + 2 * leaf_cap;
    for (int k = t; k < w; k += kTileSlots) {
        const int64_t j = b - leaf_cap + k;
        cs[k] = (j >= 0 && j + 1 < n) ? static_cast<int8_t>(common_digits(sk[j], sk[j + 1])) : int8_t(-1);
    }
    __syncthreads();
    const int64_t i = b + t;
    if (i >= n) return;
    // left slot i - 1 - dl at cs[t + leaf_cap - 1 - dl], right slot i + dr at cs[t + leaf_cap + dr]
    int kl = t + leaf_cap - 1, kr = t + leaf_cap;
    int mL = 127, mR = 127, v = -1;
    int cl = cs[kl], cr = cs[kr];
    // after step + 1 < leaf_cap moves, kl >= t and kr < t + 2 leaf_cap: both in the tile
    for (int step = 0; step < leaf_cap; ++step) {
        const int candL = min(mL, cl), candR = min(mR, cr);
        if (candL < 0 && candR < 0) { v = -1; break; }
        const bool more = step + 1 < leaf_cap;
        if (candL >= candR) {
            v = candL; mL = candL; --kl;
            if (more) cl = cs[kl];
        } else {
            v = candR; mR = candR; ++kr;
            if (more) cr = cs[kr];
        }
    }
    const int l = min(depth, v + 1);
    level[i] = static_cast<int8_t>(l);
    flag[i] = (i == 0 || static_cast<int>(cs[t + leaf_cap - 1]) < l) ? 1 : 0;
}

__global__ void k_leaf_flag_grids(const uint64_t *__restrict__ sk, int64_t n,
                                  int32_t *__restrict__ flag, int8_t *__restrict__ level,
                                  int box_level) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || (sk[i] >> 6) != (sk[i - 1] >> 6)) ? 1 : 0;
    level[i] = static_cast<int8_t>(box_level);
}

__global__ void k_leaf_write(const uint64_t *__restrict__ sk, const int8_t *__restrict__ level,
                             const int32_t *__restrict__ flag, const int32_t *__restrict__ fscan,
                             int64_t n, int kind, int32_t *__restrict__ leaf_start,
                             uint64_t *__restrict__ leaf_key, int8_t *__restrict__ leaf_level) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        if (i == 0) leaf_start[fscan[n]] = static_cast<int32_t>(n);
        if (flag[i]) {
            const int32_t L = fscan[i];
            const int l = level[i];
            leaf_start[L] = static_cast<int32_t>(i);
            leaf_level[L] = static_cast<int8_t>(l);
            const uint64_t low_bits = (kind == P2P_TREE_PARTICLES) ? 3ull * (20 - l) : 6ull;
            const uint64_t mask = (low_bits >= 64) ? 0ull : ~((1ull << low_bits) - 1ull);
            leaf_key[L] = sk[i] & mask;
        }
    }
}

// Deepest leaf level: one workgroup strides over the levels (no atomics).
__global__ __launch_bounds__(1024) void k_max_level(const int8_t *__restrict__ leaf_level,
                                                    const int32_t *__restrict__ fscan, int64_t n,
                                                    int32_t *__restrict__ out) {
    __shared__ int s_m[16];
    const int64_t L = fscan[n];
    // eight independent loads in flight per thread
    int mm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t step = 8 * static_cast<int64_t>(blockDim.x);
    int64_t i0 = threadIdx.x;
    for (; i0 + 7 * static_cast<int64_t>(blockDim.x) < L; i0 += step) {
#pragma unroll
        for (int k = 0; k < 8; ++k) mm[k] = max(mm[k], static_cast<int>(leaf_level[i0 + k * blockDim.x]));
    }
    for (int64_t i = i0; i < L; i += blockDim.x) mm[0] = max(mm[0], static_cast<int>(leaf_level[i]));
    int m = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) m = max(m, mm[k]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) r = max(r, s_m[w]);
        *out = r;
    }
}

// perm[s] = caller index of sorted slot s, and its inverse.
__global__ void k_perm_and_inverse(const int32_t *__restrict__ vals, int64_t n,
                                   int32_t *__restrict__ perm, int32_t *__restrict__ iperm) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = vals[s];
    perm[s] = i;
    iperm[i] = static_cast<int32_t>(s);
}

}  // namespace

p2p_status launch_perm_and_inverse(const int32_t *vals, int64_t n, int32_t *perm, int32_t *iperm,
                                   hipStream_t s) {
    if (n <= 0) return P2P_OK;
    k_perm_and_inverse<<<grid_for(n, 256), 256, 0, s>>>(vals, n, perm, iperm);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}


p2p_status launch_particle_keys(const double *x, const double *y, const double *z, int64_t n,
                                uint64_t *keys, int32_t *vals, int32_t *bad_flag, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    k_particle_keys<<<grid_for(n, 256), 256, 0, s>>>(x, y, z, n, keys, vals, bad_flag);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_grid_keys(const int32_t *d_n_side, const int64_t *d_point_off, int32_t n_grids,
                            int bits, int64_t n, uint64_t *keys, int32_t *vals, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    k_grid_keys<<<grid_for(n, 256), 256, 0, s>>>(d_n_side, d_point_off, n_grids, bits, n, keys, vals);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_leaf_levels(const uint64_t *skeys, int64_t n, int kind, int depth, int leaf_cap,
                              uint8_t *pair_common, int8_t *level, int32_t *flags, hipStream_t s) {
    if (n <= 0) return P2P_OK;
    if (kind == P2P_TREE_PARTICLES && leaf_cap > 0 && leaf_cap <= 64) {
        k_leaf_level_ballot<<<grid_for(n, 256), 256, 0, s>>>(skeys, n, depth, leaf_cap, level, flags);
    } else if (kind == P2P_TREE_PARTICLES && leaf_cap > 0 && leaf_cap <= kTileCap) {
        k_leaf_level_tile<<<grid_for(n, kTileSlots), kTileSlots, kTileSlots + 2 * leaf_cap, s>>>(
            skeys, n, depth, leaf_cap, level, flags);
    } else if (kind == P2P_TREE_PARTICLES) {
        if (n > 1) {
            k_pair_common<<<grid_for(n - 1, 256), 256, 0, s>>>(skeys, n, pair_common);
            P2P_LAUNCH_CHECK();
        }
        k_leaf_level_particles<<<grid_for(n, 256), 256, 0, s>>>(pair_common, n, depth, leaf_cap,
                                                                level, flags);
    } else {
        k_leaf_flag_grids<<<grid_for(n, 256), 256, 0, s>>>(skeys, n, flags, level, depth);
    }
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_leaf_write(const uint64_t *skeys, const int8_t *level, const int32_t *flags,
                             const int32_t *flag_scan, int64_t n, int kind, int32_t *leaf_start,
                             uint64_t *leaf_key, int8_t *leaf_level, int32_t *max_level,
                             hipStream_t s) {
    if (n <= 0) return P2P_OK;
    k_leaf_write<<<grid_for(n, 256), 256, 0, s>>>(skeys, level, flags, flag_scan, n, kind,
                                                  leaf_start, leaf_key, leaf_level);
    P2P_LAUNCH_CHECK();
    k_max_level<<<1, 1024, 0, s>>>(leaf_level, flag_scan, n, max_level);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace p2p
