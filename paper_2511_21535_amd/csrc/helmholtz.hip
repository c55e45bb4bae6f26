// Near-field Helmholtz on regular grids, VALU path (Sec. 5.1; FP64, and
// right-hand-side counts the matrix-core kernels do not take).
//
// Grid leaves are boxes of 4x4x4 points.  One wavefront owns one target box:
// lane l holds the target at local Morton index l.  For each near box B the
// 64 sources are uniform across the wave (scalar loads), and the kernel value
// depends only on the integer squared index distance dd in 0..147 between
// target and source, so G comes from a per-instance table of 148 complex
// values in LDS, built in FP64 and rounded to the working precision
// (the precomputed interaction patterns of the DBIM case, Sec. 5.1).  Entry
// dd = 0 is zero, which removes the self term without a test.  With
// e = l_t - 4 o (o = box offset of B) and source local coordinates
// (sx, sy, sz) in 0..3, dd = (e_x - sx)^2 + (e_y - sy)^2 + (e_z - sz)^2; the
// per-axis squares are precomputed per box, so each pair costs one integer
// add, one LDS read and four FMAs.  The near boxes of a target box are dealt
// to the four wavefronts of its workgroup (box e to wave e % 4), which gives
// four times the waves to hide the scalar loads of the sources; the four
// partial sums meet in LDS.
#include <type_traits>

#include "p2p_internal.h"

namespace p2p {
namespace {

constexpr double kPi = 3.14159265358979323846;

template <class C>
__global__ void k_green_tables(const double *__restrict__ h, const double *__restrict__ k,
                               int32_t n_grids, C *__restrict__ table) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n_grids) * kTableLen) return;
    const int g = static_cast<int>(t / kTableLen), dd = static_cast<int>(t % kTableLen);
    C v;
    if (dd == 0) {
        v.x = 0;
        v.y = 0;
    } else {
        const double r = h[g] * sqrt(static_cast<double>(dd));
        const double a = 1.0 / (4.0 * kPi * r);
        double sn, cs;
        sincos(k[g] * r, &sn, &cs);
        v.x = static_cast<decltype(v.x)>(cs * a);
        v.y = static_cast<decltype(v.y)>(sn * a);
    }
    table[t] = v;
}

template <class C> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };

__device__ inline int lane_axis(int l, int axis) {
    return ((l >> axis) & 1) | (((l >> (axis + 3)) & 1) << 1);
}

constexpr int kHWaves = 4;

// COMP (FP32 payload): each near box's 64-term FP32 partial sum is added into
// an FP64 per-target sum; otherwise all terms accumulate in the payload's type.
template <class C, bool RED, bool CONJ, bool ONE, bool COMP>
__global__ __launch_bounds__(64 * kHWaves) void k_helmholtz(
    int64_t L, int key_bits, int32_t nrhs, const int32_t *__restrict__ leaf_start,
    const uint64_t *__restrict__ leaf_key, const int32_t *__restrict__ perm,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, const int64_t *__restrict__ red_row, const C *__restrict__ src,
    const C *__restrict__ tables, C *__restrict__ u) {
    using R = typename Real<C>::T;
    using P = typename std::conditional<COMP, double2, C>::type;   // partial sums across waves
    __shared__ C s_tab[kTableLen];
    __shared__ P s_part[kHWaves][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t A = blockIdx.x;
    const uint64_t local_mask = (1ull << (3 * key_bits)) - 1ull;
    const uint64_t kA = leaf_key[A];
    const int g = static_cast<int>(kA >> (3 * key_bits));
    const C *__restrict__ table = tables + static_cast<int64_t>(g) * kTableLen;
    for (int i = threadIdx.x; i < kTableLen; i += 64 * kHWaves) s_tab[i] = table[i];
    __syncthreads();

    const uint64_t lA = kA & local_mask;
    const int ax = static_cast<int>(p2pd::compact3(lA)), ay = static_cast<int>(p2pd::compact3(lA >> 1)),
              az = static_cast<int>(p2pd::compact3(lA >> 2));
    const int lt[3] = {lane_axis(lane, 0), lane_axis(lane, 1), lane_axis(lane, 2)};
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
    const char *tab = reinterpret_cast<const char *>(s_tab);

    const int64_t stride = ONE ? 1 : nrhs;
    for (int32_t r = 0; r < (ONE ? 1 : nrhs); ++r) {
        R ur = 0, ui = 0;
        double cr = 0.0, ci = 0.0;
        for (int64_t e = e0 + wv; e < e1; e += kHWaves) {
            const int32_t B = nbr_idx[e];
            const uint64_t lB = leaf_key[B] & local_mask;
            const int o[3] = {(static_cast<int>(p2pd::compact3(lB)) - ax) / 4,
                              (static_cast<int>(p2pd::compact3(lB >> 1)) - ay) / 4,
                              (static_cast<int>(p2pd::compact3(lB >> 2)) - az) / 4};
            // redundant rows: the entry's place in A's segment (box grain) or
            // in the segment of A's tile (red_row, tile grain)
            const int64_t row0 = RED ? (red_row ? red_row[e] : red_start[A] + 64 * (e - e0)) : leaf_start[B];
            const C *__restrict__ qb = src + row0 * stride + r;
            int sq[3][4];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int ed = lt[d] - 4 * o[d];
#pragma unroll
                for (int k = 0; k < 4; ++k) sq[d][k] = (ed - k) * (ed - k) * static_cast<int>(sizeof(C));
            }
            int sxy[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) sxy[k] = sq[0][k & 3] + sq[1][k >> 2];
#pragma unroll
            for (int ls = 0; ls < 64; ++ls) {
                const int kx = (ls & 1) | ((ls >> 2) & 2);
                const int ky = ((ls >> 1) & 1) | ((ls >> 3) & 2);
                const int kz = ((ls >> 2) & 1) | ((ls >> 4) & 2);
                const C gv = *reinterpret_cast<const C *>(tab + sxy[kx + 4 * ky] + sq[2][kz]);
                const C q = qb[static_cast<int64_t>(ls) * stride];
                // conj(A conj(q)) = conj(G) q: negate the imaginary part of G instead of q and u
                const R gi = CONJ ? -gv.y : gv.y;
                ur = fma(gv.x, q.x, ur);
                ur = fma(-gi, q.y, ur);
                ui = fma(gv.x, q.y, ui);
                ui = fma(gi, q.x, ui);
            }
            if constexpr (COMP) {
                cr += static_cast<double>(ur);
                ci += static_cast<double>(ui);
                ur = 0;
                ui = 0;
            }
        }
        P part;
        if constexpr (COMP) {
            part.x = cr;
            part.y = ci;
        } else {
            part.x = ur;
            part.y = ui;
        }
        s_part[wv][lane] = part;
        __syncthreads();
        if (wv == 0) {
            P out = s_part[0][lane];
#pragma unroll
            for (int q = 1; q < kHWaves; ++q) {
                out.x += s_part[q][lane].x;
                out.y += s_part[q][lane].y;
            }
            const int64_t i = perm[leaf_start[A] + lane];
            C o;
            o.x = static_cast<R>(out.x);
            o.y = static_cast<R>(out.y);
            u[i * stride + r] = o;
        }
        __syncthreads();
    }
}

}  // namespace

p2p_status launch_green_tables(const double *d_h, const double *d_k, int32_t n_grids, bool fp64,
                               void *table, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(n_grids) * kTableLen;
    if (fp64)
        k_green_tables<double2><<<grid_for(n, 256), 256, 0, s>>>(d_h, d_k, n_grids,
                                                                static_cast<double2 *>(table));
    else
        k_green_tables<float2><<<grid_for(n, 256), 256, 0, s>>>(d_h, d_k, n_grids,
                                                               static_cast<float2 *>(table));
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

template <class C, bool RED, bool CONJ, bool COMP>
static void launch_helm_c(const HelmholtzArgs &a, hipStream_t s) {
    if (a.nrhs == 1)
        k_helmholtz<C, RED, CONJ, true, COMP><<<static_cast<unsigned>(a.L), 64 * kHWaves, 0, s>>>(
            a.L, a.key_bits, a.nrhs, a.leaf_start, a.leaf_key, a.perm, a.nbr_start, a.nbr_idx,
            a.red_start, a.red_row, static_cast<const C *>(a.src), static_cast<const C *>(a.table),
            static_cast<C *>(a.u));
    else
        k_helmholtz<C, RED, CONJ, false, COMP><<<static_cast<unsigned>(a.L), 64 * kHWaves, 0, s>>>(
            a.L, a.key_bits, a.nrhs, a.leaf_start, a.leaf_key, a.perm, a.nbr_start, a.nbr_idx,
            a.red_start, a.red_row, static_cast<const C *>(a.src), static_cast<const C *>(a.table),
            static_cast<C *>(a.u));
}

template <class C, bool RED, bool CONJ>
static void launch_helm_t(const HelmholtzArgs &a, hipStream_t s) {
    if (a.comp && std::is_same<C, float2>::value)
        launch_helm_c<C, RED, CONJ, true>(a, s);
    else
        launch_helm_c<C, RED, CONJ, false>(a, s);
}

p2p_status launch_helmholtz(const HelmholtzArgs &a, bool redundant, bool fp64, hipStream_t s) {
    if (a.L <= 0) return P2P_OK;
    const bool cj = a.conj != 0;
    if (fp64) {
        if (redundant) { if (cj) launch_helm_t<double2, true, true>(a, s); else launch_helm_t<double2, true, false>(a, s); }
        else { if (cj) launch_helm_t<double2, false, true>(a, s); else launch_helm_t<double2, false, false>(a, s); }
    } else {
        if (redundant) { if (cj) launch_helm_t<float2, true, true>(a, s); else launch_helm_t<float2, true, false>(a, s); }
        else { if (cj) launch_helm_t<float2, false, true>(a, s); else launch_helm_t<float2, false, false>(a, s); }
    }
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace p2p
