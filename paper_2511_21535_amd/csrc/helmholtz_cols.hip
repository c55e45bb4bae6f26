// Single right-hand side of the near-field Helmholtz sum on the matrix cores,
// FP32 and FP64 (the dense regular case of Sec. 5.1 with one right-hand side),
// the target boxes taken as the columns of the product.  Kept in a file of its
// own: it is compiled with the matrix accumulators in ordinary vector
// registers (-amdgpu-mfma-vgpr-form), so the FP32 kernel's per-offset FP64
// flush reads them without a copy out of the accumulation registers.
#include <algorithm>

#include "p2p_internal.h"

namespace p2p {
namespace {

// Single right-hand side on matrix cores: the target boxes become the columns
// of the product.  For a tile of up to 16 boxes b_0..b_15 of one instance,
//     U (64 x 16) = sum_o G_o (64 x 64) Q_o (64 x 16),
// column j of Q_o holding the 64 sources of the box at offset o from b_j (a
// zero column where b_j has no such neighbour, at the faces of the grid), so
// every column of an instruction shares the one G_o.  v_mfma_f32_16x16x4f32,
// complex as three real products; lane l supplies A[l%16][l/16] and
// B[l/16][l%16], and accumulator register r of lane l holds row 4 (l/16) + r,
// column l%16.  A workgroup of 4 wavefronts owns a tile; wave w takes the
// offsets o = w, w + 4, ... for all 64 targets (four row tiles, 12
// instructions per k-step of 4 sources) with a deep operand prefetch, and the
// four partial products are summed through LDS at the end.  The workgroup
// first maps every (offset, column) to the first row of its sources -- the
// sorted rows of the neighbour box (gather) or its place in the target's
// segment (redundant) -- from the tile's near lists, which are one contiguous
// run of the CSR.
constexpr int kColBoxes = kHelmColBoxes;
constexpr int kColWaves = 4;
static_assert(kColWaves == 4, "wave w finishes row tile w of the four");
// prefetch distances of the G and Q operands, in k-steps (the buffer rotation
// runs on across offsets of 16 k-steps each)
constexpr int kColPrefG = 3;
constexpr int kColPrefQ = 7;

// The column tile of workgroup b: its first box A0, box count cnt, G table tab
// and 1/h of its instance (sc in float; sc64 in double from inl.iscale64 or
// inst_h, when inst_h or the inline parameters are given).
__device__ inline void col_tile(int key_bits, const int32_t *__restrict__ tiles, const HelmInline &inl,
                                const uint64_t *__restrict__ leaf_key, const int32_t *__restrict__ inst_table,
                                const float *__restrict__ inst_scale, const double *__restrict__ inst_h, int32_t b,
                                int32_t &A0, int32_t &cnt, int32_t &tab, float &sc, double &sc64) {
    sc64 = 1.0;
    if (inl.n_grids > 0) {
        int32_t tf = 0, lf = 0, lf1 = 0;
        tab = 0;
        sc = 1.f;
#pragma unroll
        for (int i = 0; i < kInlineGrids; ++i)
            if (i < inl.n_grids && b >= inl.tile_first[i]) {
                tf = inl.tile_first[i];
                lf = inl.leaf_first[i];
                lf1 = inl.leaf_first[i + 1];
                tab = inl.itab[i];
                sc = inl.iscale[i];
                sc64 = inl.iscale64[i];
            }
        A0 = lf + kColBoxes * (b - tf);
        cnt = min(kColBoxes, lf1 - A0);
    } else {
        A0 = tiles[2 * b];
        cnt = tiles[2 * b + 1];
        const int g = static_cast<int>(leaf_key[A0] >> (3 * key_bits));
        tab = inst_table ? inst_table[g] : 0;
        sc = inst_scale ? inst_scale[g] : 1.f;
        if (inst_h) sc64 = 1.0 / inst_h[g];
    }
}

// The (offset, column) map of a tile in LDS: the first source row of every
// (offset, column) from the tile's near lists (one contiguous run of the CSR;
// -1 where the column has no such neighbour), and each column's first sorted
// target row.
struct ColMap {
    int64_t row[27][kColBoxes];
    int64_t nstart[kColBoxes + 1];
    uint64_t key[kColBoxes];      // local Morton key of each column's box
    int64_t rstart[kColBoxes];    // its segment start (redundant layout, box grain)
    int32_t tstart[kColBoxes];    // its first sorted target row
};

// Fills m; called by the whole workgroup (64 kColWaves threads), ends with a
// barrier.  Each column's list start, key, segment start and first target row
// come in one round of loads; then the entries, two per thread with their
// loads issued together: at most 27 per box, so one round covers a tile.
template <bool RED>
__device__ void col_map(ColMap &m, int key_bits, int32_t A0, int32_t cnt, const int32_t *__restrict__ leaf_start,
                        const uint64_t *__restrict__ leaf_key, const int64_t *__restrict__ nbr_start,
                        const int32_t *__restrict__ nbr_idx, const int64_t *__restrict__ red_start,
                        const int64_t *__restrict__ red_row) {
    const int tid = threadIdx.x;
    const uint64_t local_mask = (1ull << (3 * key_bits)) - 1ull;
    for (int i = tid; i < 27 * kColBoxes; i += 64 * kColWaves) m.row[i / kColBoxes][i % kColBoxes] = -1;
    if (tid <= cnt) {
        // all four loads in flight at once (thread cnt only needs the list end)
        const int32_t a = A0 + min(tid, cnt - 1);
        const int64_t ns = nbr_start[A0 + tid];
        const uint64_t key = leaf_key[a];
        const int64_t rs = (RED && !red_row) ? red_start[a] : 0;
        const int32_t ts = leaf_start[a];
        m.nstart[tid] = ns;
        if (tid < cnt) {
            m.key[tid] = key & local_mask;
            m.rstart[tid] = rs;
            m.tstart[tid] = ts;
        }
    }
    __syncthreads();
    const int64_t e_lo = m.nstart[0], e_hi = m.nstart[cnt];
    constexpr int kT = 64 * kColWaves;
    for (int64_t e0 = e_lo + tid; e0 < e_hi; e0 += 2 * kT) {
        int64_t ev[2] = {e0, e0 + kT};
        int32_t Bv[2];
        uint64_t lB[2];
        int64_t rv[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) Bv[p] = nbr_idx[ev[p] < e_hi ? ev[p] : e0];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            lB[p] = leaf_key[Bv[p]] & local_mask;
            rv[p] = RED ? (red_row ? red_row[ev[p] < e_hi ? ev[p] : e0] : 0) : static_cast<int64_t>(leaf_start[Bv[p]]);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int64_t e = ev[p];
            if (e >= e_hi) break;
            int j = 0;
            while (j + 1 < cnt && m.nstart[j + 1] <= e) ++j;
            const uint64_t lA = m.key[j];
            const int ox = (static_cast<int>(p2pd::compact3(lB[p])) - static_cast<int>(p2pd::compact3(lA))) / 4;
            const int oy =
                (static_cast<int>(p2pd::compact3(lB[p] >> 1)) - static_cast<int>(p2pd::compact3(lA >> 1))) / 4;
            const int oz =
                (static_cast<int>(p2pd::compact3(lB[p] >> 2)) - static_cast<int>(p2pd::compact3(lA >> 2))) / 4;
            const int o = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
            m.row[o][j] = (RED && !red_row) ? m.rstart[j] + 64 * (e - m.nstart[j]) : rv[p];
        }
    }
    __syncthreads();
}

// H workgroups per tile as in k_helm_mfma_cols64 below (H = 2 on grids with at
// most half as many tiles as CUs): each part then stores its result, the FP64
// sums or the FP32 tile, in sorted order to parts[p][.] as double2, and
// k_join_parts adds the two in double and rounds the sum once.
template <bool RED, bool CONJ, bool COMP, int H>
__global__ __launch_bounds__(64 * kColWaves) void k_helm_mfma_cols(
    int key_bits, const int32_t *__restrict__ tiles, HelmInline inl, const int32_t *__restrict__ leaf_start,
    const uint64_t *__restrict__ leaf_key, const int32_t *__restrict__ perm,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, const int64_t *__restrict__ red_row, const float2 *__restrict__ src,
    const float2 *__restrict__ blocks, const float2 *__restrict__ zeros, const int32_t *__restrict__ inst_table,
    const float *__restrict__ inst_scale, float2 *__restrict__ u, double2 *__restrict__ parts, int64_t n) {
    typedef float floatx4 __attribute__((ext_vector_type(4)));
    constexpr int VW = kColWaves * H;              // waves sharing a tile's offsets
    constexpr int NSL = (27 + VW - 1) / VW;        // offset slots per wave
    __shared__ ColMap sm;
    // the partial sums of every wave for every row tile (wave w finishes row
    // tile w): FP32 tiles, or FP64 sums under COMP
    __shared__ floatx4 s_red[COMP ? 1 : kColWaves][4][2][64];
    __shared__ double s_redd[COMP ? kColWaves * 4 * 2 * 4 * 64 : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // the tile: its first box, its box count, the G table and 1/h of its instance
    int32_t A0, cnt, tab;
    float sc;
    double sc64;
    const int32_t b = static_cast<int32_t>(blockIdx.x) / H, part = static_cast<int32_t>(blockIdx.x) % H;
    col_tile(key_bits, tiles, inl, leaf_key, inst_table, inst_scale, nullptr, b, A0, cnt, tab, sc, sc64);
    col_map<RED>(sm, key_bits, A0, cnt, leaf_start, leaf_key, nbr_start, nbr_idx, red_start, red_row);

    const int li = lane & 15, kq = lane >> 4;
    const int vw = part * kColWaves + w;
    const float2 *__restrict__ gbase = blocks + static_cast<int64_t>(tab) * (27 * 4096);
    // Every instruction of the k-step loop that is not a matrix product or a load
    // takes issue cycles from the matrix cores (the vector and matrix units share
    // them), so the loop holds only the five additions of the three-product form
    // (Re Q + Im Q and the four Re G +- Im G, cheaper than a G layout that stores
    // the sums: that doubles the G reads from L2, measured slower): the G base of
    // an offset is uniform (scalar registers, a lane adds only its fixed offset),
    // a lane's four row-tile values of G sit in one 32-byte run (the single-RHS
    // layout), a column without the neighbour reads 64 zero rows instead of being
    // masked, and the signs of the three-product form are applied once per offset
    // or at the end, from the three accumulators.  Lane (k, i) reads, at k-step kk, G_o[source
    // 4 kk + k][targets i, 16 + i, 32 + i, 48 + i] and Q[source 4 kk + k] of
    // column i.
    // Wave w takes the offsets o = w + 4 idx, idx = 0..6 (H = 1), without a
    // branch: the one slot past the 27 offsets (wave 3's last) and every column
    // without the neighbour read the zero rows, which add exact zeros.  A
    // branch would let the compiler sink the next offset's prefetch loads below
    // it and drain the load pipeline at every offset.
    const int goff = (kq * 16 + li) * 4;
    auto ptrs = [&](int idx, const float2 *&Gs, const float2 *&Qp) {
        const int o = vw + VW * idx;
        const int64_t row = o < 27 ? sm.row[o][li] : int64_t(-1);
        Gs = gbase + (o < 27 ? o : 0) * 4096;
        Qp = (row >= 0 ? src + row : zeros) + kq;
    };
    int32_t dst[4] = {0, 0, 0, 0};
    // The complex product in three real products (the 3M form, as in the
    // multi-RHS kernel): pa = sum Re G Re Q, pb = sum Im G Im Q,
    // pc = sum (Re G + Im G)(Re Q + Im Q); U = G Q: Re = pa - pb,
    // Im = pc - pa - pb.  With CONJ (conj G) pc takes Re G - Im G:
    // Re = pa + pb, Im = pc - pa + pb.
    floatx4 pa[4], pb[4], pc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) pa[rt] = pb[rt] = pc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto re_of = [&](int rt, int r) { return CONJ ? pa[rt][r] + pb[rt][r] : pa[rt][r] - pb[rt][r]; };
    auto im_of = [&](int rt, int r) {
        return CONJ ? pc[rt][r] - pa[rt][r] + pb[rt][r] : pc[rt][r] - pa[rt][r] - pb[rt][r];
    };
    // COMP: FP64 per-target sums of the per-offset FP32 partial products
    constexpr int CN = COMP ? 4 : 1;
    double cr[4][CN], ci[4][CN];
    if constexpr (COMP) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) cr[rt][r] = ci[rt][r] = 0.0;
    }
    // fresh: the first k-step of an offset under COMP starts from zero
    auto mma = [&](const float2 (&gv)[4], const float2 q, bool fresh) {
        const floatx4 zero = floatx4{0.f, 0.f, 0.f, 0.f};
        const float qs = q.x + q.y;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const float gs = CONJ ? gv[rt].x - gv[rt].y : gv[rt].x + gv[rt].y;
            pa[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[rt].x, q.x, fresh ? zero : pa[rt], 0, 0, 0);
            pb[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[rt].y, q.y, fresh ? zero : pb[rt], 0, 0, 0);
            pc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(gs, qs, fresh ? zero : pc[rt], 0, 0, 0);
        }
    };
    {
        // The wave's 7 x 16 k-steps, unrolled as one sequence (a loop would carry
        // the twelve accumulators across its back edge, which the register
        // allocator pays for with copies on every iteration).  G is read from
        // L2 and issued kColPrefG steps ahead; the Q rows (the redundant layout
        // streams from HBM) kColPrefQ steps ahead, each step's G loads issued
        // before its Q load so that waiting for a step's G never waits for a
        // younger Q.  Scheduling barriers keep the loads where they are.
        const float2 *Gs[NSL], *Qs[NSL];
#pragma unroll
        for (int idx = 0; idx < NSL; ++idx) ptrs(idx, Gs[idx], Qs[idx]);
        constexpr int NS = NSL * 16;
        float2 gbuf[kColPrefG + 1][4], qbuf[kColPrefQ + 1];
        auto load_g = [&](int st) {
            const float4 *g4 = reinterpret_cast<const float4 *>(Gs[st / 16] + (st % 16) * 256 + goff);
            const float4 lo = g4[0], hi = g4[1];
            float2(&gv)[4] = gbuf[st % (kColPrefG + 1)];
            gv[0] = make_float2(lo.x, lo.y);
            gv[1] = make_float2(lo.z, lo.w);
            gv[2] = make_float2(hi.x, hi.y);
            gv[3] = make_float2(hi.z, hi.w);
        };
        auto load_q = [&](int st) { qbuf[st % (kColPrefQ + 1)] = Qs[st / 16][(st % 16) * 4]; };
#pragma unroll
        for (int st = 0; st < kColPrefG; ++st) load_g(st);
#pragma unroll
        for (int st = 0; st < kColPrefQ; ++st) load_q(st);
        // the caller-order rows of the four targets this lane stores at the end
        // (row tile w), loaded behind the first operands so that no k-step waits
        // for them
        if (li < cnt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int32_t sr = sm.tstart[li] + 16 * w + 4 * kq + r;
                dst[r] = H == 1 ? perm[sr] : sr;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // (two nested unrolled loops: one loop of 112 steps exceeds the unroller's limit)
#pragma unroll
        for (int idx = 0; idx < NSL; ++idx) {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int st = idx * 16 + kk;
                if (st + kColPrefG < NS) load_g(st + kColPrefG);
                if (st + kColPrefQ < NS) load_q(st + kColPrefQ);
                __builtin_amdgcn_sched_barrier(0);
                mma(gbuf[st % (kColPrefG + 1)], qbuf[st % (kColPrefQ + 1)], COMP && kk == 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (COMP) {
                // each offset's 64-term FP32 partial product into the FP64 sums
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        cr[rt][r] += static_cast<double>(re_of(rt, r));
                        ci[rt][r] += static_cast<double>(im_of(rt, r));
                    }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    floatx4 ur[4], ui[4];
    if constexpr (!COMP) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ur[rt][r] = re_of(rt, r);
                ui[rt][r] = im_of(rt, r);
            }
    }
    // Wave w finishes row tile w: every wave leaves its partial sums in LDS,
    // then wave w adds the four waves' partials of row tile w in wave order
    // 0..3 and stores its targets.
    auto red_at = [&](int q, int rt, int im, int r) -> double & {
        return s_redd[(((q * 4 + rt) * 2 + im) * 4 + r) * 64 + lane];
    };
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        if constexpr (COMP) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                red_at(w, rt, 0, r) = cr[rt][r];
                red_at(w, rt, 1, r) = ci[rt][r];
            }
        } else {
            s_red[w][rt][0][lane] = ur[rt];
            s_red[w][rt][1][lane] = ui[rt];
        }
    }
    __syncthreads();
    if (li < cnt) {
        if constexpr (COMP) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double tr = red_at(0, w, 0, r), ti = red_at(0, w, 1, r);
#pragma unroll
                for (int q = 1; q < kColWaves; ++q) {
                    tr += red_at(q, w, 0, r);
                    ti += red_at(q, w, 1, r);
                }
                if constexpr (H == 1)
                    u[dst[r]] = make_float2(static_cast<float>(tr * sc), static_cast<float>(ti * sc));
                else
                    parts[part * n + dst[r]] = make_double2(tr * sc, ti * sc);
            }
        } else {
            floatx4 fr = s_red[0][w][0][lane], fi = s_red[0][w][1][lane];
#pragma unroll
            for (int q = 1; q < kColWaves; ++q) {
                fr += s_red[q][w][0][lane];
                fi += s_red[q][w][1][lane];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if constexpr (H == 1)
                    u[dst[r]] = make_float2(fr[r] * sc, fi[r] * sc);
                else
                    parts[part * n + dst[r]] = make_double2(fr[r] * sc, fi[r] * sc);
            }
        }
    }
}


// FP64 single right-hand side on the FP64 matrix cores: the same product as
// k_helm_mfma_cols with v_mfma_f64_16x16x4f64 (four real products per
// complex one, all sums in double; G blocks in double2, same layout).  Lane l
// supplies A[l%16][l/16] and B[l/16][l%16] as in FP32, but accumulator
// register r of lane l holds row l/16 + 4 r (rows interleaved), column l%16.
// A tile's 27 offsets may be shared by H workgroups (H = 2 on grids with at
// most half as many tiles as CUs, so that twice the CUs work): wave w of part
// p takes offsets o = 4 p + w + 4 H idx.  With H = 2 each part stores its
// result in sorted order to parts[p][.] (coalesced), and k_join_parts64 adds
// part 0 and part 1 and scatters the sum to the caller's order (FP64 atomic
// additions at the scattered caller rows took 7 us more on a 48^3 grid).
template <bool RED, bool CONJ, int H>
__global__ __launch_bounds__(64 * kColWaves) void k_helm_mfma_cols64(
    int key_bits, const int32_t *__restrict__ tiles, HelmInline inl, const int32_t *__restrict__ leaf_start,
    const uint64_t *__restrict__ leaf_key, const int32_t *__restrict__ perm,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int64_t *__restrict__ red_start, const int64_t *__restrict__ red_row, const double2 *__restrict__ src,
    const double2 *__restrict__ blocks, const double2 *__restrict__ zeros, const int32_t *__restrict__ inst_table,
    const double *__restrict__ inst_h, double2 *__restrict__ u, double2 *__restrict__ parts, int64_t n) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    constexpr int VW = kColWaves * H;              // waves sharing a tile's offsets
    constexpr int NSL = (27 + VW - 1) / VW;        // offset slots per wave
    __shared__ ColMap sm;
    __shared__ double s_red[kColWaves][4][2][4][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int32_t b = static_cast<int32_t>(blockIdx.x) / H, part = static_cast<int32_t>(blockIdx.x) % H;
    int32_t A0, cnt, tab;
    float sc;
    double sc64;
    col_tile(key_bits, tiles, inl, leaf_key, inst_table, nullptr, inst_h, b, A0, cnt, tab, sc, sc64);
    col_map<RED>(sm, key_bits, A0, cnt, leaf_start, leaf_key, nbr_start, nbr_idx, red_start, red_row);

    const int li = lane & 15, kq = lane >> 4;
    const double2 *__restrict__ gbase = blocks + static_cast<int64_t>(tab) * (27 * 4096);
    // lane (kq, li) reads, at k-step kk, G_o[source 4 kk + kq][targets li, 16 + li, 32 + li, 48 + li]
    // (one 64-byte run) and Q[source 4 kk + kq] of column li; the slots past the 27
    // offsets and absent neighbours read the zero rows
    const int goff = (kq * 16 + li) * 4;
    const int vw = part * kColWaves + w;
    auto ptrs = [&](int idx, const double2 *&Gs, const double2 *&Qp) {
        const int o = vw + VW * idx;
        const int64_t row = o < 27 ? sm.row[o][li] : int64_t(-1);
        Gs = gbase + (o < 27 ? o : 0) * 4096;
        Qp = (row >= 0 ? src + row : zeros) + kq;
    };
    int32_t dst[4] = {0, 0, 0, 0};
    // three real products per complex one, as in the FP32 kernel: pa = sum Re G Re Q,
    // pb = sum Im G Im Q, pc = sum (Re G +- Im G)(Re Q + Im Q), the sums formed per k-step
    f64x4 pa[4], pb[4], pc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) pa[rt] = pb[rt] = pc[rt] = f64x4{0.0, 0.0, 0.0, 0.0};
    {
        const double2 *Gs[NSL], *Qs[NSL];
#pragma unroll
        for (int idx = 0; idx < NSL; ++idx) ptrs(idx, Gs[idx], Qs[idx]);
        constexpr int NS = NSL * 16;
        double2 gbuf[kColPrefG + 1][4], qbuf[kColPrefQ + 1];
        auto load_g = [&](int st) {
            const double2 *g = Gs[st / 16] + (st % 16) * 256 + goff;
            double2(&gv)[4] = gbuf[st % (kColPrefG + 1)];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) gv[rt] = g[rt];
        };
        auto load_q = [&](int st) { qbuf[st % (kColPrefQ + 1)] = Qs[st / 16][(st % 16) * 4]; };
#pragma unroll
        for (int st = 0; st < kColPrefG; ++st) load_g(st);
#pragma unroll
        for (int st = 0; st < kColPrefQ; ++st) load_q(st);
        // the rows of the four targets this lane stores at the end: caller-order
        // rows, or sorted rows in this part's half of `parts`
        if (li < cnt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int32_t sr = sm.tstart[li] + 16 * w + kq + 4 * r;
                dst[r] = H == 1 ? perm[sr] : sr;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int idx = 0; idx < NSL; ++idx) {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int st = idx * 16 + kk;
                if (st + kColPrefG < NS) load_g(st + kColPrefG);
                if (st + kColPrefQ < NS) load_q(st + kColPrefQ);
                __builtin_amdgcn_sched_barrier(0);
                const double2(&gv)[4] = gbuf[st % (kColPrefG + 1)];
                const double2 q = qbuf[st % (kColPrefQ + 1)];
                const double qs = q.x + q.y;
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const double gs = CONJ ? gv[rt].x - gv[rt].y : gv[rt].x + gv[rt].y;
                    pa[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[rt].x, q.x, pa[rt], 0, 0, 0);
                    pb[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[rt].y, q.y, pb[rt], 0, 0, 0);
                    pc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(gs, qs, pc[rt], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // U = G Q: Re = pa - pb, Im = pc - pa - pb; with CONJ (conj G): Re = pa + pb,
    // Im = pc - pa + pb.  Wave w finishes row tile w from the four waves' partials, in
    // wave order.
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s_red[w][rt][0][r][lane] = CONJ ? pa[rt][r] + pb[rt][r] : pa[rt][r] - pb[rt][r];
            s_red[w][rt][1][r][lane] = CONJ ? pc[rt][r] - pa[rt][r] + pb[rt][r] : pc[rt][r] - pa[rt][r] - pb[rt][r];
        }
    __syncthreads();
    if (li < cnt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double tr = s_red[0][w][0][r][lane], ti = s_red[0][w][1][r][lane];
#pragma unroll
            for (int q = 1; q < kColWaves; ++q) {
                tr += s_red[q][w][0][r][lane];
                ti += s_red[q][w][1][r][lane];
            }
            if constexpr (H == 1)
                u[dst[r]] = make_double2(tr * sc64, ti * sc64);
            else
                parts[part * n + dst[r]] = make_double2(tr * sc64, ti * sc64);
        }
    }
}

// u[perm[s]] = parts[0][s] + parts[1][s] for every sorted row s, added in
// double and rounded once.
__global__ void k_join_parts(const double2 *__restrict__ parts, const int32_t *__restrict__ perm, int64_t n,
                             float2 *__restrict__ u) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 a = parts[i], b = parts[n + i];
    u[perm[i]] = make_float2(static_cast<float>(a.x + b.x), static_cast<float>(a.y + b.y));
}

// u[perm[s]] = parts[0][s] + parts[1][s] for every sorted row s.
__global__ void k_join_parts64(const double2 *__restrict__ parts, const int32_t *__restrict__ perm, int64_t n,
                               double2 *__restrict__ u) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 a = parts[i], b = parts[n + i];
    u[perm[i]] = make_double2(a.x + b.x, a.y + b.y);
}

}  // namespace

int32_t helmholtz_cols_tiles(const p2p_grid *grids, int32_t n_grids, int32_t *tiles) {
    int64_t first = 0;
    int32_t t = 0;
    for (int32_t g = 0; g < n_grids; ++g) {
        const int64_t nb = static_cast<int64_t>(grids[g].n_side / 4) * (grids[g].n_side / 4) * (grids[g].n_side / 4);
        for (int64_t b = 0; b < nb; b += kColBoxes, ++t) {
            if (tiles) {
                tiles[2 * t] = static_cast<int32_t>(first + b);
                tiles[2 * t + 1] = static_cast<int32_t>(std::min<int64_t>(kColBoxes, nb - b));
            }
        }
        first += nb;
    }
    return t;
}

template <bool R, bool C, int H>
static void launch_cols64(const HelmholtzMfmaArgs &a, const int32_t *tiles, const HelmInline &inl, int32_t n_tiles,
                          hipStream_t s) {
    k_helm_mfma_cols64<R, C, H><<<static_cast<unsigned>(n_tiles) * H, 64 * kColWaves, 0, s>>>(
        a.key_bits, tiles, inl, a.leaf_start, a.leaf_key, a.perm, a.nbr_start, a.nbr_idx, a.red_start, a.red_row,
        reinterpret_cast<const double2 *>(a.src), reinterpret_cast<const double2 *>(a.blocks),
        reinterpret_cast<const double2 *>(a.zeros), a.inst_table, a.inst_h, reinterpret_cast<double2 *>(a.u), a.parts,
        a.n);
}

p2p_status launch_helmholtz_mfma_cols(const HelmholtzMfmaArgs &a, const int32_t *tiles, const HelmInline &inl,
                                      int32_t n_tiles, bool redundant, bool fp64, hipStream_t s) {
    if (n_tiles <= 0) return P2P_OK;
    if (fp64) {
        int dev = 0, cus = 0;
        P2P_HIP(hipGetDevice(&dev));
        P2P_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const bool split = 2 * static_cast<int64_t>(n_tiles) <= cus && a.parts;
        const bool cj = a.conj != 0;
#define P2P_MF64(H)                                                                  \
    if (redundant) { if (cj) launch_cols64<true, true, H>(a, tiles, inl, n_tiles, s);    \
                     else launch_cols64<true, false, H>(a, tiles, inl, n_tiles, s); }    \
    else { if (cj) launch_cols64<false, true, H>(a, tiles, inl, n_tiles, s);             \
           else launch_cols64<false, false, H>(a, tiles, inl, n_tiles, s); }
        if (split) { P2P_MF64(2) } else { P2P_MF64(1) }
#undef P2P_MF64
        P2P_LAUNCH_CHECK();
        if (split) {
            k_join_parts64<<<grid_for(a.n, 256), 256, 0, s>>>(a.parts, a.perm, a.n, reinterpret_cast<double2 *>(a.u));
            P2P_LAUNCH_CHECK();
        }
        return P2P_OK;
    }
    int dev = 0, cus = 0;
    P2P_HIP(hipGetDevice(&dev));
    P2P_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const bool split = 2 * static_cast<int64_t>(n_tiles) <= cus && a.parts;
#define P2P_MFC3(R, C, M, H)                                                                            \
    k_helm_mfma_cols<R, C, M, H><<<static_cast<unsigned>(n_tiles) * H, 64 * kColWaves, 0, s>>>(        \
        a.key_bits, tiles, inl, a.leaf_start, a.leaf_key, a.perm, a.nbr_start, a.nbr_idx, a.red_start, a.red_row, a.src, \
        a.blocks, a.zeros, a.inst_table, a.inst_scale, a.u, a.parts, a.n)
#define P2P_MFC2(R, C, M) if (split) P2P_MFC3(R, C, M, 2); else P2P_MFC3(R, C, M, 1)
#define P2P_MFC(R, C) if (a.comp) { P2P_MFC2(R, C, true); } else { P2P_MFC2(R, C, false); }
    const bool cj = a.conj != 0;
    if (redundant) { if (cj) { P2P_MFC(true, true); } else { P2P_MFC(true, false); } }
    else { if (cj) { P2P_MFC(false, true); } else { P2P_MFC(false, false); } }
#undef P2P_MFC
#undef P2P_MFC2
#undef P2P_MFC3
    P2P_LAUNCH_CHECK();
    if (split) {
        k_join_parts<<<grid_for(a.n, 256), 256, 0, s>>>(a.parts, a.perm, a.n, a.u);
        P2P_LAUNCH_CHECK();
    }
    return P2P_OK;
}

}  // namespace p2p
