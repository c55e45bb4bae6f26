// Locality metric inputs (a12; Definition 1 of the paper, Sec. 3.4).
//
// Per target leaf A: D_A = number of maximal runs of consecutive leaf ids in
// nbr(A) (leaves occupy contiguous memory in id order, so each run is one
// contiguous block the gather layout reads); the redundant layout reads one
// segment, D = 1.  Also summed: S = sum_A sum_{B in nbr(A)} occ(B) (entries
// of the redundant layout) and P = sum_A occ(A) sum_{B in nbr(A)} occ(B)
// (ordered near pairs before removing the N self pairs).
#include "p2p_internal.h"

namespace p2p {
namespace {

__global__ void k_locality_stats(const int32_t *__restrict__ leaf_start,
                                 const int64_t *__restrict__ nbr_start,
                                 const int32_t *__restrict__ nbr_idx, int64_t L,
                                 unsigned long long *__restrict__ sums) {
    const int64_t A = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long runs = 0, seg = 0, pairs = 0;
    if (A < L) {
        int32_t prev = -2;
        for (int64_t e = nbr_start[A]; e < nbr_start[A + 1]; ++e) {
            const int32_t B = nbr_idx[e];
            if (B != prev + 1) ++runs;
            prev = B;
            seg += static_cast<unsigned long long>(leaf_start[B + 1] - leaf_start[B]);
        }
        pairs = seg * static_cast<unsigned long long>(leaf_start[A + 1] - leaf_start[A]);
    }
    // wave reduction, then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
        runs += __shfl_down(runs, o, 64);
        seg += __shfl_down(seg, o, 64);
        pairs += __shfl_down(pairs, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&sums[0], runs);
        atomicAdd(&sums[1], seg);
        atomicAdd(&sums[2], pairs);
    }
}

}  // namespace

p2p_status launch_locality_stats(const int32_t *leaf_start, const int64_t *nbr_start,
                                 const int32_t *nbr_idx, int64_t L, unsigned long long *sums,
                                 hipStream_t s) {
    if (L <= 0) return P2P_OK;
    k_locality_stats<<<grid_for(L, 256), 256, 0, s>>>(leaf_start, nbr_start, nbr_idx, L, sums);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace p2p
