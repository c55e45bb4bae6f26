// Multi-RHS near-field Helmholtz on FP32 matrix cores in one persistent
// launch over every box of every grid instance (the dense regular case of
// Sec. 5.1, many instances batched).
//
// For target box b (64 points) and R right-hand sides:
//     U_b (64 x R) = sum_{o in near offsets} G_o (64 x 64) Q_{b+o} (64 x R),
// a dense complex contraction.  On a regular grid G_o depends only on the box
// offset o (27 values) and on k h, so the 27 blocks are built once per call
// in FP64 for unit spacing (G scales as 1/h) and shared by all boxes of all
// instances with the same k h; the scale 1/h is applied when U is stored.
//
// One wavefront owns one target box and a chunk of 32*TJ right-hand sides.
// The complex product runs as four real v_mfma_f32_32x32x2f32 per 32x32
// tile: Re U += Re G Re Q - Im G Im Q, Im U += Re G Im Q + Im G Re Q.  Per
// k-step (2 sources) a lane loads one complex G entry per row tile and one
// complex Q entry per column tile; G is stored source-major, [o][s][t], and
// Q row-major, [s][rhs], so both loads are contiguous across 32 lanes.
// Lane layouts of the instruction: A[i][k] from lane k*32 + i, B[k][j] from
// lane k*32 + j, and accumulator register r of lane l holds row
// 8 (r/4) + 4 (l/32) + r%4, column l%32.
//
// Work distribution: waves take (box, RHS chunk) items in tree order from
// eight atomic counters, one per XCD, each over a contiguous eighth of the
// items, and exit when every eighth is exhausted.
//
// The G blocks can be held in several identical copies (the block-level
// pattern redundancy of the paper's electromagnetic case, Sec. 5.1.2, there
// with a redundancy factor RF): the workgroups of one XCD then read different
// copies, spreading the pattern loads over more L2 lines and channels.
#include <algorithm>

#include "p2p_internal.h"

namespace p2p {
namespace {

typedef __amdgpu_buffer_rsrc_t Rsrc;
// A raw buffer descriptor over [p, p + bytes): dword 3 holds the 32-bit data
// format that untyped (raw) buffer loads expect on this target.
__device__ inline Rsrc buffer_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}

typedef float floatx16 __attribute__((ext_vector_type(16)));
constexpr double kPi = 3.14159265358979323846;

// G(t, o, s, i) = e^{i kh sqrt(dd)} / (4 pi sqrt(dd)), dd = |l_i - (l_s + 4 o)|^2, zero for
// dd = 0, for table t, offset o = (ox+1) + 3 (oy+1) + 9 (oz+1), source s and target i (l_*
// are local Morton coordinates).  Multi-RHS layout: float4 (Re G, Im G, Re G + Im G,
// Re G - Im G) at [t][c][o][s][i], identical for every copy c (the three-product form of
// the complex product reads the sum, its conjugate the difference; both are formed in
// double and rounded once).  Single-RHS (COLS) layout: float2 at [t][o][s][i % 16][i / 16],
// the four row tiles of a target column next to each other, so a lane reads the four it
// needs in one 32-byte run, followed by 64 zero entries (the source rows of an absent
// neighbour); the FP64 single-RHS path keeps the same layout in double2.
__global__ void k_green_blocks(const double *__restrict__ kh_dev, HelmInline inl, int32_t n_tables,
                               int32_t copies, bool cols, bool f64, void *__restrict__ out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = 27 * 64 * 64, total = per * n_tables * copies;
    if (t >= total + (cols ? 64 : 0)) return;
    if (t >= total) {
        if (f64)
            static_cast<double2 *>(out)[t] = make_double2(0.0, 0.0);
        else
            static_cast<float2 *>(out)[t] = make_float2(0.f, 0.f);
        return;
    }
    const int tab = static_cast<int>(t / (per * copies));
    double khv = 0.0;
    if (inl.n_grids > 0) {
        // compile-time indices only, so the argument array stays in the kernel arguments
#pragma unroll
        for (int i = 0; i < kInlineGrids; ++i)
            if (i == tab) khv = inl.kh[i];
    } else {
        khv = kh_dev[tab];
    }
    const int rem = static_cast<int>(t % per);
    const int o = rem / 4096, s = (rem / 64) % 64, i = rem % 64;
    const int od[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
    int dd = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int li = ((i >> d) & 1) | (((i >> (d + 3)) & 1) << 1);
        const int ls = ((s >> d) & 1) | (((s >> (d + 3)) & 1) << 1);
        const int diff = li - (ls + 4 * od[d]);
        dd += diff * diff;
    }
    double gr = 0.0, gi = 0.0;
    if (dd > 0) {
        const double r = sqrt(static_cast<double>(dd));
        const double a = 1.0 / (4.0 * kPi * r);
        double sn, cs;
        sincos(khv * r, &sn, &cs);
        gr = cs * a;
        gi = sn * a;
    }
    const int64_t at = static_cast<int64_t>(tab) * per + o * 4096 + s * 64 + (i % 16) * 4 + i / 16;
    if (cols && f64)
        static_cast<double2 *>(out)[at] = make_double2(gr, gi);
    else if (cols)
        static_cast<float2 *>(out)[at] = make_float2(static_cast<float>(gr), static_cast<float>(gi));
    else
        static_cast<float4 *>(out)[t] = make_float4(static_cast<float>(gr), static_cast<float>(gi),
                                                    static_cast<float>(gr + gi), static_cast<float>(gr - gi));
}

__global__ void k_zero_counter(int32_t *c, int n) {
    if (static_cast<int>(threadIdx.x) < n) c[threadIdx.x] = 0;
}

// COMP: the accumulators restart from zero for every near box, and each
// box's 64-term FP32 partial product is added into FP64 per-target sums (the
// per-target accumulation in double of FP32 partial sums); otherwise the
// products of all near boxes accumulate in FP32.
// M3: the complex product takes three real products per tile instead of four
// (the 3M form): A = Re G Re Q, B = Im G Im Q, C = (Re G + Im G)(Re Q + Im Q), then
// Re U = A - B and Im U = C - A - B; with CONJ (conj G), C takes Re G - Im G and
// Re U = A + B, Im U = C - A + B.  One addition per Q value and k-step (Re Q +
// Im Q); G brings its sum and difference with it.  Otherwise four products:
// Re U = Re G Re Q - Im G Im Q, Im U = Re G Im Q + Im G Re Q.
template <bool RED, bool CONJ, int TJ, bool COMP, bool M3>
__device__ __forceinline__ void helm_mfma_body(
    int64_t L, int key_bits, int32_t nrhs, const int32_t *__restrict__ leaf_start,
    const uint64_t *__restrict__ leaf_key, const int32_t *__restrict__ perm,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, const int64_t *__restrict__ red_row, const float2 *__restrict__ src,
    const float4 *__restrict__ blocks, int32_t copies, const int32_t *__restrict__ inst_table,
    const float *__restrict__ inst_scale, int32_t *__restrict__ counter, float2 *__restrict__ u) {
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5, col = lane & 31;
    const uint64_t local_mask = (1ull << (3 * key_bits)) - 1ull;
    const int chunks = nrhs / (32 * TJ);
    const int64_t items = L * chunks;

    // The items (box, RHS chunk), boxes in tree order, form eight contiguous
    // slices, one per XCD (workgroups are dispatched to the XCDs round-robin,
    // blockIdx.x % 8): the boxes one XCD runs at a time are neighbours, whose
    // near fields overlap in its L2.  A wave whose slice is exhausted takes
    // items from the next slices in turn; counters only grow, so a slice found
    // exhausted stays so and every wave ends after at most eight misses.
    const int xcd = static_cast<int>(blockIdx.x & 7);
    int sl = 0;   // lane 0: slices found exhausted
    for (;;) {
        int item = -1;
        if (lane == 0) {
            for (; sl < 8; ++sl) {
                const int x = (xcd + sl) & 7;
                const int64_t lo = items * x / 8, hi = items * (x + 1) / 8;
                const int64_t it = lo + atomicAdd(&counter[x], 1);
                if (it < hi) {
                    item = static_cast<int>(it);
                    break;
                }
            }
        }
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
        if (item < 0) break;
        const int64_t A = item / chunks;
        const int rhs0 = (item % chunks) * 32 * TJ;
        const uint64_t kA = leaf_key[A];
        const int g = static_cast<int>(kA >> (3 * key_bits));
        // the workgroups of one XCD (w % 8 equal) spread over the copies
        const int64_t copy = (blockIdx.x >> 3) % copies;
        const float4 *__restrict__ gbase = blocks + (static_cast<int64_t>(inst_table[g]) * copies + copy) * (27 * 4096);
        const uint64_t lA = kA & local_mask;
        const int ax = static_cast<int>(p2pd::compact3(lA)), ay = static_cast<int>(p2pd::compact3(lA >> 1)),
                  az = static_cast<int>(p2pd::compact3(lA >> 2));
        const int64_t e0 = nbr_start[A];
        const int ne = static_cast<int>(nbr_start[A + 1] - e0);

        // lane e (< ne) works out the operand offsets of near box e once: the
        // G block of its offset and its first Q row; the k-loop reads them
        // back with readlane, so no memory access sits between boxes
        int my_goff = 0, my_row_lo = 0, my_row_hi = 0;
        if (lane < ne) {
            const int32_t B = nbr_idx[e0 + lane];
            const uint64_t lB = leaf_key[B] & local_mask;
            const int ox = (static_cast<int>(p2pd::compact3(lB)) - ax) / 4;
            const int oy = (static_cast<int>(p2pd::compact3(lB >> 1)) - ay) / 4;
            const int oz = (static_cast<int>(p2pd::compact3(lB >> 2)) - az) / 4;
            my_goff = ((ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)) * 4096;
            // redundant rows: the entry's place in A's segment (box grain) or
            // in the segment of A's tile (red_row, tile grain)
            const int64_t row0 = RED ? (red_row ? red_row[e0 + lane] : red_start[A] + 64 * static_cast<int64_t>(lane))
                                     : leaf_start[B];
            my_row_lo = static_cast<int>(row0 & 0xffffffff);
            my_row_hi = static_cast<int>(row0 >> 32);
        }
        // Operands through buffer loads: a descriptor per near box over its G
        // block and its 64 source rows (scalar registers), a lane offset fixed
        // for the whole item and a per-k-step scalar offset, so that no k-step
        // spends vector instructions on address arithmetic.  Reads beyond a
        // descriptor's range would return zeros; the offsets stay inside it.
        auto box_ptrs = [&](int e, Rsrc &Gp, Rsrc &Qp) {
            const int goff = __builtin_amdgcn_readlane(my_goff, e);
            const int64_t row0 = (static_cast<int64_t>(__builtin_amdgcn_readlane(my_row_hi, e)) << 32) |
                                 static_cast<uint32_t>(__builtin_amdgcn_readlane(my_row_lo, e));
            Gp = buffer_rsrc(gbase + goff, 4096 * static_cast<int>(sizeof(float4)));
            Qp = buffer_rsrc(src + row0 * nrhs + rhs0, (64 * nrhs - rhs0) * static_cast<int>(sizeof(float2)));
        };
        const int vg = (half * 64 + col) * static_cast<int>(sizeof(float4));
        const int vq = (half * nrhs + col) * static_cast<int>(sizeof(float2));

        // M3: pa = A, pb = B, pc = C; otherwise ur = pa (Re U), ui = pb (Im U)
        constexpr int NC = M3 ? TJ : 1;
        floatx16 pa[2][TJ], pb[2][TJ], pc[2][NC];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int b = 0; b < TJ; ++b) pa[a][b] = pb[a][b] = floatx16{0};
#pragma unroll
            for (int b = 0; b < NC; ++b) pc[a][b] = floatx16{0};
        }
        auto re_of = [&](int a, int b, int r) -> float {
            if constexpr (M3) return CONJ ? pa[a][b][r] + pb[a][b][r] : pa[a][b][r] - pb[a][b][r];
            else return pa[a][b][r];
        };
        auto im_of = [&](int a, int b, int r) -> float {
            if constexpr (M3)
                return CONJ ? pc[a][b % NC][r] - pa[a][b][r] + pb[a][b][r] : pc[a][b % NC][r] - pa[a][b][r] - pb[a][b][r];
            else return pb[a][b][r];
        };
        // FP64 per-target sums of the per-box partial products (COMP)
        constexpr int CN = COMP ? 16 : 1;
        double cr[2][TJ][CN], ci[2][TJ][CN];
        if constexpr (COMP) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < TJ; ++b)
#pragma unroll
                    for (int r = 0; r < 16; ++r) cr[a][b][r] = ci[a][b][r] = 0.0;
        }

        const int qstep = 2 * nrhs * static_cast<int>(sizeof(float2));   // two source rows per k-step
        auto load = [&](Rsrc Gp, Rsrc Qp, int kk, float4 (&gv)[2], float2 (&qv)[TJ]) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
                gv[a] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                                                       Gp, vg + 32 * a * static_cast<int>(sizeof(float4)), kk * 2048, 0));
#pragma unroll
            for (int b = 0; b < TJ; ++b)
                qv[b] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                                       Qp, vq + 32 * b * static_cast<int>(sizeof(float2)), kk * qstep, 0));
        };
        // fresh: the first k-step of a box under COMP starts from zero accumulators
        auto mma = [&](const float4 (&gv)[2], const float2 (&qv)[TJ], bool fresh) {
            const floatx16 zero = floatx16{0};
            if constexpr (M3) {
                float qs[TJ];
#pragma unroll
                for (int b = 0; b < TJ; ++b) qs[b] = qv[b].x + qv[b].y;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float gs = CONJ ? gv[a].w : gv[a].z;
#pragma unroll
                    for (int b = 0; b < TJ; ++b) {
                        pa[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(gv[a].x, qv[b].x, fresh ? zero : pa[a][b], 0, 0, 0);
                        pb[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(gv[a].y, qv[b].y, fresh ? zero : pb[a][b], 0, 0, 0);
                        pc[a][b % NC] =
                            __builtin_amdgcn_mfma_f32_32x32x2f32(gs, qs[b], fresh ? zero : pc[a][b % NC], 0, 0, 0);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float gr = gv[a].x, gi = CONJ ? -gv[a].y : gv[a].y;
#pragma unroll
                    for (int b = 0; b < TJ; ++b) {
                        pa[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(gr, qv[b].x, fresh ? zero : pa[a][b], 0, 0, 0);
                        pb[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(gr, qv[b].y, fresh ? zero : pb[a][b], 0, 0, 0);
                        pa[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-gi, qv[b].y, pa[a][b], 0, 0, 0);
                        pb[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(gi, qv[b].x, pb[a][b], 0, 0, 0);
                    }
                }
            }
        };

        // four operand buffers in rotation: the loads of k-step kk + 3 are issued
        // while step kk runs, across box boundaries (the last box prefetches
        // its own first steps again, harmlessly)
        Rsrc Gc, Gn, Qc, Qn;
        box_ptrs(0, Gc, Qc);
        float4 gbuf[4][2];
        float2 qbuf[4][TJ];
        load(Gc, Qc, 0, gbuf[0], qbuf[0]);
        load(Gc, Qc, 1, gbuf[1], qbuf[1]);
        load(Gc, Qc, 2, gbuf[2], qbuf[2]);
        for (int e = 0; e < ne; ++e) {
            box_ptrs(e + 1 < ne ? e + 1 : e, Gn, Qn);
#pragma unroll
            for (int kk = 0; kk < 32; ++kk) {
                const int ks = kk + 3;
                if (ks < 32)
                    load(Gc, Qc, ks, gbuf[ks & 3], qbuf[ks & 3]);
                else
                    load(Gn, Qn, ks - 32, gbuf[ks & 3], qbuf[ks & 3]);
                // keep the prefetch where it is: without the barrier the
                // scheduler sinks each load down to its first use, and every
                // k-step then waits out a full L2 round trip
                __builtin_amdgcn_sched_barrier(0);
                mma(gbuf[kk & 3], qbuf[kk & 3], COMP && kk == 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (COMP) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < TJ; ++b)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            cr[a][b][r] += static_cast<double>(re_of(a, b, r));
                            ci[a][b][r] += static_cast<double>(im_of(a, b, r));
                        }
            }
            Gc = Gn;
            Qc = Qn;
        }
        const float sc = inst_scale[g];
        const int32_t t0 = leaf_start[A];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = 32 * a + 8 * (r / 4) + 4 * half + (r % 4);
                const int64_t row = static_cast<int64_t>(perm[t0 + i]) * nrhs + rhs0 + col;
#pragma unroll
                for (int b = 0; b < TJ; ++b) {
                    if constexpr (COMP)
                        u[row + 32 * b] = make_float2(static_cast<float>(cr[a][b][r] * sc),
                                                      static_cast<float>(ci[a][b][r] * sc));
                    else
                        u[row + 32 * b] = make_float2(re_of(a, b, r) * sc, im_of(a, b, r) * sc);
                }
            }
    }
}

#define P2P_HELM_MFMA_PARAMS                                                                            \
    int64_t L, int key_bits, int32_t nrhs, const int32_t *__restrict__ leaf_start,                      \
        const uint64_t *__restrict__ leaf_key, const int32_t *__restrict__ perm,                        \
        const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,                     \
        const int64_t *__restrict__ red_start, const int64_t *__restrict__ red_row,                     \
        const float2 *__restrict__ src, const float4 *__restrict__ blocks, int32_t copies,              \
        const int32_t *__restrict__ inst_table, const float *__restrict__ inst_scale,                   \
        int32_t *__restrict__ counter, float2 *__restrict__ u
#define P2P_HELM_MFMA_ARGS                                                                              \
    L, key_bits, nrhs, leaf_start, leaf_key, perm, nbr_start, nbr_idx, red_start, red_row, src, blocks, \
        copies, inst_table, inst_scale, counter, u

// The product form of each variant: three real products, except 64 right-hand
// sides per wave with FP64 sums, whose 128 doubles per lane of sums leave no
// room for a third set of accumulators.
template <int TJ, bool COMP>
constexpr bool kM3 = !(TJ == 2 && COMP);

// Two waves per SIMD: 32 right-hand sides per wave in FP32.
template <bool RED, bool CONJ, int TJ, bool COMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_helm_mfma(P2P_HELM_MFMA_PARAMS) {
    helm_mfma_body<RED, CONJ, TJ, COMP, kM3<TJ, COMP>>(P2P_HELM_MFMA_ARGS);
}

// One wave per SIMD: 64 right-hand sides per wave, or FP64 sums (their doubles
// per lane do not fit beside the accumulators at two waves per SIMD).
template <bool RED, bool CONJ, int TJ, bool COMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1))) void k_helm_mfma_wide(
    P2P_HELM_MFMA_PARAMS) {
    helm_mfma_body<RED, CONJ, TJ, COMP, kM3<TJ, COMP>>(P2P_HELM_MFMA_ARGS);
}

}  // namespace

p2p_status launch_green_blocks(const double *d_kh, const HelmInline &inl, int32_t n_tables, int32_t copies,
                               bool cols, bool f64, void *blocks, hipStream_t s) {
    if (cols && copies != 1) return fail(P2P_EINVAL, "internal: the single-RHS G layout has one copy");
    if (f64 && !cols) return fail(P2P_EINVAL, "internal: FP64 G blocks exist in the single-RHS layout only");
    const int64_t n = static_cast<int64_t>(n_tables) * copies * 27 * 4096 + (cols ? 64 : 0);
    k_green_blocks<<<grid_for(n, 256), 256, 0, s>>>(d_kh, inl, n_tables, copies, cols, f64, blocks);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}


template <bool RED, bool CONJ, int TJ, bool COMP>
static void launch_mfma_t(const HelmholtzMfmaArgs &a, unsigned grid, unsigned block, hipStream_t s) {
    const float4 *g4 = reinterpret_cast<const float4 *>(a.blocks);
    if constexpr (TJ == 2 || COMP)
        k_helm_mfma_wide<RED, CONJ, TJ, COMP><<<grid, block, 0, s>>>(
            a.L, a.key_bits, a.nrhs, a.leaf_start, a.leaf_key, a.perm, a.nbr_start, a.nbr_idx,
            a.red_start, a.red_row, a.src, g4, a.copies, a.inst_table, a.inst_scale, a.counter, a.u);
    else
        k_helm_mfma<RED, CONJ, TJ, COMP><<<grid, block, 0, s>>>(
            a.L, a.key_bits, a.nrhs, a.leaf_start, a.leaf_key, a.perm, a.nbr_start, a.nbr_idx,
            a.red_start, a.red_row, a.src, g4, a.copies, a.inst_table, a.inst_scale, a.counter, a.u);
}

p2p_status launch_helmholtz_mfma(const HelmholtzMfmaArgs &a, bool redundant, int waves_per_wg,
                                 int wg_per_cu, int rhs_tile, hipStream_t s) {
    if (a.L <= 0) return P2P_OK;
    int dev = 0, cus = 0;
    P2P_HIP(hipGetDevice(&dev));
    P2P_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    k_zero_counter<<<1, 64, 0, s>>>(a.counter, 8);
    P2P_LAUNCH_CHECK();
    const unsigned block = 64u * static_cast<unsigned>(waves_per_wg);
    const unsigned grid = static_cast<unsigned>(cus) * static_cast<unsigned>(wg_per_cu);
    const bool cj = a.conj != 0;
    const int TJ = (rhs_tile == 64) ? 2 : 1;
#define P2P_MF(R, C, T) \
    (a.comp ? launch_mfma_t<R, C, T, true>(a, grid, block, s) : launch_mfma_t<R, C, T, false>(a, grid, block, s))
    if (TJ == 2) {
        if (redundant) { if (cj) P2P_MF(true, true, 2); else P2P_MF(true, false, 2); }
        else { if (cj) P2P_MF(false, true, 2); else P2P_MF(false, false, 2); }
    } else {
        if (redundant) { if (cj) P2P_MF(true, true, 1); else P2P_MF(true, false, 1); }
        else { if (cj) P2P_MF(false, true, 1); else P2P_MF(false, false, 1); }
    }
#undef P2P_MF
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace p2p
