// Device-wide exclusive scan and stable LSD radix sort of (uint64 key, int32
// value) pairs.  Both are plain data-movement primitives used by tree
// binning, near-list construction and the restructure step.
#include "p2p_internal.h"

namespace p2p {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;   // 2048
constexpr int64_t kScanFusedBlocks = 4096;            // n up to 8M in two launches

// Exclusive scan of one value per thread across a 256-thread block.
// Returns the thread's exclusive prefix; *total receives the block sum.
template <class T>
__device__ T block_exclusive_scan(T v, T *lds /*[kScanBlock/64]*/, T *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    T wave_off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / 64; ++w) {
        T s = lds[w];
        if (w < wave) wave_off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wave_off + x - v;
}

template <class TI, class TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const TI *__restrict__ in, int64_t n,
                                                            TO *__restrict__ partial) {
    __shared__ TO lds[kScanBlock / 64];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    TO s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += static_cast<TO>(in[base + i]);
    TO tot;
    block_exclusive_scan<TO>(s, lds, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Scans partial[0..nb) in place (exclusive) with a single block; partial[nb] = total.
template <class TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_partials(TO *partial, int64_t nb) {
    __shared__ TO lds[kScanBlock / 64];
    TO carry = 0;
    for (int64_t c = 0; c < nb; c += kScanTile) {
        int64_t base = c + threadIdx.x * kScanItems;
        TO v[kScanItems];
        TO s = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = (base + i < nb) ? partial[base + i] : TO(0);
            s += v[i];
        }
        TO tot;
        TO pre = block_exclusive_scan<TO>(s, lds, &tot) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < nb) partial[base + i] = pre;
            pre += v[i];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nb] = carry;
}

// Down-sweep.  The block's offset is partial[blockIdx.x] when the partials
// were scanned by k_scan_partials (FUSED == false); with FUSED the block sums
// the raw block totals partial[0 .. blockIdx.x) itself (one launch fewer, for
// grids of up to kScanFusedBlocks blocks), and partial == nullptr means a
// single block with offset 0.
template <class TI, class TO, bool FUSED>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const TI *in, int64_t n,
                                                          const TO *__restrict__ partial,
                                                          int64_t nb, TO *out) {
    __shared__ TO lds[kScanBlock / 64];
    TO off = 0, tot;
    if (FUSED && partial) {
        for (int64_t i = threadIdx.x; i < blockIdx.x; i += kScanBlock) off += partial[i];
        block_exclusive_scan<TO>(off, lds, &tot);
        off = tot;
    } else if (!FUSED) {
        off = partial[blockIdx.x];
    }
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    TO v[kScanItems];
    TO s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? static_cast<TO>(in[base + i]) : TO(0);
        s += v[i];
    }
    TO pre = block_exclusive_scan<TO>(s, lds, &tot) + off;
    // every read of `in` by this block happened before the barrier inside the scan
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) {
        if (FUSED && blockIdx.x == nb - 1) out[n] = off + tot;
        if (!FUSED && blockIdx.x == 0) out[n] = partial[nb];
    }
}

template <class TO>
__global__ void k_scan_empty(TO *out) { out[0] = 0; }

}  // namespace

size_t scan_ws_elems(int64_t n) { return static_cast<size_t>((n + kScanTile - 1) / kScanTile) + 2; }

template <class TI, class TO>
p2p_status exclusive_scan(const TI *in, TO *out, int64_t n, TO *scratch, hipStream_t s) {
    if (n <= 0) {
        k_scan_empty<TO><<<1, 1, 0, s>>>(out);
        P2P_LAUNCH_CHECK();
        return P2P_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    const unsigned g = static_cast<unsigned>(nb);
    if (nb == 1) {
        k_scan_down<TI, TO, true><<<1, kScanBlock, 0, s>>>(in, n, nullptr, nb, out);
        P2P_LAUNCH_CHECK();
    } else if (nb <= kScanFusedBlocks) {
        k_scan_reduce<TI, TO><<<g, kScanBlock, 0, s>>>(in, n, scratch);
        P2P_LAUNCH_CHECK();
        k_scan_down<TI, TO, true><<<g, kScanBlock, 0, s>>>(in, n, scratch, nb, out);
        P2P_LAUNCH_CHECK();
    } else {
        k_scan_reduce<TI, TO><<<g, kScanBlock, 0, s>>>(in, n, scratch);
        P2P_LAUNCH_CHECK();
        k_scan_partials<TO><<<1, kScanBlock, 0, s>>>(scratch, nb);
        P2P_LAUNCH_CHECK();
        k_scan_down<TI, TO, false><<<g, kScanBlock, 0, s>>>(in, n, scratch, nb, out);
        P2P_LAUNCH_CHECK();
    }
    return P2P_OK;
}

template p2p_status exclusive_scan<int32_t, int32_t>(const int32_t *, int32_t *, int64_t, int32_t *,
                                                     hipStream_t);
template p2p_status exclusive_scan<int32_t, int64_t>(const int32_t *, int64_t *, int64_t, int64_t *,
                                                     hipStream_t);
template p2p_status exclusive_scan<int64_t, int64_t>(const int64_t *, int64_t *, int64_t, int64_t *,
                                                     hipStream_t);
template p2p_status exclusive_scan<uint32_t, uint32_t>(const uint32_t *, uint32_t *, int64_t,
                                                       uint32_t *, hipStream_t);

// ------------------------------------------------------------------ sort --
namespace {

constexpr int kSortBlock = 256;                 // 4 waves
constexpr int kSortChunks = 16;                 // chunks of 64 keys per wave
constexpr int kSortWaveKeys = 64 * kSortChunks; // 1024
constexpr int kSortTile = 4 * kSortWaveKeys;    // 4096 keys per block

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                           int64_t n, int shift,
                                                           uint32_t *__restrict__ hist,
                                                           int64_t ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
#pragma unroll 4
    for (int i = 0; i < kSortTile / kSortBlock; ++i) {
        int64_t idx = base + i * kSortBlock + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one 8-bit digit.  Each wave ranks its 1024 keys in order,
// chunk by chunk: lanes holding the same digit are found with 8 ballots, the
// lane's rank among them is a popcount below its lane, and a per-wave digit
// counter in LDS carries the running count from chunk to chunk.  Wave
// counters are then scanned across the 4 waves and across the 256 digits,
// which gives every key its position in the tile sorted by digit (stable).
// The tile is rearranged in LDS into that order and written out in order, so
// the keys of one digit leave as one contiguous, coalesced run.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offs,
    int64_t ntiles) {
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t dstart[256];     // first tile position of each digit
    __shared__ uint32_t s_w[4];
    __shared__ uint64_t s_key[kSortTile];
    __shared__ int32_t s_val[kSortTile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * 256; i += kSortBlock) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t tbase = static_cast<int64_t>(blockIdx.x) * kSortTile;
    const int64_t wbase = tbase + wave * kSortWaveKeys;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t key[kSortChunks];
    int32_t val[kSortChunks];
    uint32_t loc[kSortChunks];
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c) {
        const int64_t idx = wbase + c * 64 + lane;
        const bool valid = idx < n;
        key[c] = valid ? kin[idx] : 0ull;
        val[c] = valid ? vin[idx] : 0;
        const uint32_t d = static_cast<uint32_t>(key[c] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = __popcll(peers & below);
        const uint32_t base = valid ? cnt[wave][d] : 0u;
        if (valid && rank == 0) cnt[wave][d] = base + static_cast<uint32_t>(__popcll(peers));
        loc[c] = base + rank;
    }
    __syncthreads();
    // per digit (thread = digit): exclusive scan over the waves, and the digit's total
    uint32_t tot = 0;
    for (int w = 0; w < 4; ++w) {
        const uint32_t t = cnt[w][threadIdx.x];
        cnt[w][threadIdx.x] = tot;
        tot += t;
    }
    // exclusive scan of the digit totals across the 256 threads
    uint32_t inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t woff = 0;
    for (int w = 0; w < wave; ++w) woff += s_w[w];
    dstart[threadIdx.x] = woff + inc - tot;
    __syncthreads();
    // rearrange the tile in LDS by digit
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c) {
        const int64_t idx = wbase + c * 64 + lane;
        if (idx < n) {
            const uint32_t d = static_cast<uint32_t>(key[c] >> shift) & 255u;
            const uint32_t pos = dstart[d] + cnt[wave][d] + loc[c];
            s_key[pos] = key[c];
            s_val[pos] = val[c];
        }
    }
    __syncthreads();
    // write out in tile order: position i of digit d goes to offs[d] + (i - dstart[d])
    const int tile_n = static_cast<int>(min<int64_t>(kSortTile, n - tbase));
    for (int i = threadIdx.x; i < tile_n; i += kSortBlock) {
        const uint64_t k = s_key[i];
        const uint32_t d = static_cast<uint32_t>(k >> shift) & 255u;
        const int64_t pos = static_cast<int64_t>(offs[static_cast<int64_t>(d) * ntiles + blockIdx.x]) +
                            (i - static_cast<int64_t>(dstart[d]));
        kout[pos] = k;
        vout[pos] = s_val[i];
    }
}

__global__ void k_copy_pairs(const uint64_t *__restrict__ ks, const int32_t *__restrict__ vs,
                             uint64_t *__restrict__ kd, int32_t *__restrict__ vd, int64_t n) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

}  // namespace

size_t radix_hist_elems(int64_t n) {
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int64_t m = 256 * (ntiles > 0 ? ntiles : 1);
    return static_cast<size_t>(m + 1) + scan_ws_elems(m);
}

p2p_status radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp,
                            int64_t n, int key_bits, uint32_t *hist_scratch, hipStream_t s) {
    if (n <= 1) return P2P_OK;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    const int64_t m = 256 * ntiles;
    uint32_t *hist = hist_scratch;
    uint32_t *scan_tmp = hist_scratch + m + 1;
    uint64_t *ka = keys, *kb = keys_tmp;
    int32_t *va = vals, *vb = vals_tmp;
    for (int shift = 0; shift < key_bits; shift += 8) {
        k_radix_hist<<<static_cast<unsigned>(ntiles), kSortBlock, 0, s>>>(ka, n, shift, hist, ntiles);
        P2P_LAUNCH_CHECK();
        P2P_TRY((exclusive_scan<uint32_t, uint32_t>(hist, hist, m, scan_tmp, s)));
        k_radix_scatter<<<static_cast<unsigned>(ntiles), kSortBlock, 0, s>>>(ka, va, kb, vb, n, shift,
                                                                            hist, ntiles);
        P2P_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        k_copy_pairs<<<grid_for(n, 256), 256, 0, s>>>(ka, va, keys, vals, n);
        P2P_LAUNCH_CHECK();
    }
    return P2P_OK;
}

}  // namespace p2p
