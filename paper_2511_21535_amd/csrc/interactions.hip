// Per-interaction redundant layout for gravity: the thread-level redundancy of
// the paper's stellar-dynamics case (Sec. 5.2.1), beside the box-grain layout
// of restructure.hip.
//
// One record per near-list entry e = (A, B): a header row (occ_A, occ_B, A, B
// as integers), A's rows (the targets), then B's rows (the sources).  Every
// record is self-contained, so the evaluation takes one wavefront per record
// with no shared state; its pair sums go to result rows of its own (the
// duplicated results of the paper's design), and a second pass sums each
// target's rows over the records of its leaf (the update).  Compared with the
// box grain, the layout stores every target E2 times more and every result
// E2 times, in exchange for independent, fine-grained work items.
#include <type_traits>

#include "p2p_internal.h"

namespace p2p {
namespace {

constexpr int kRecLanes = 16;

__device__ inline float rsq_f32(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ inline void put(float4 *d, const float4 &v) {
    if constexpr (NT) {
        const nt_f4 t = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(t, reinterpret_cast<nt_f4 *>(d));
    } else {
        *d = v;
    }
}
template <bool NT>
__device__ inline void put(Row4d *d, const Row4d &v) {
    if constexpr (NT) {
        const nt_d2 a = {v.x, v.y}, b = {v.z, v.w};
        __builtin_nontemporal_store(a, reinterpret_cast<nt_d2 *>(d));
        __builtin_nontemporal_store(b, reinterpret_cast<nt_d2 *>(d) + 1);
    } else {
        *d = v;
    }
}

// rec_len[e] = 1 + occ_A + occ_B and tgt_len[e] = occ_A for the entries of
// leaf A (16 lanes per leaf).  Either output may be null.
__global__ __launch_bounds__(256) void k_record_lengths(const int32_t *__restrict__ leaf_start,
                                                        const int64_t *__restrict__ nbr_start,
                                                        const int32_t *__restrict__ nbr_idx, int64_t L,
                                                        int32_t *__restrict__ rec_len,
                                                        int32_t *__restrict__ tgt_len) {
    const int sub = threadIdx.x % kRecLanes;
    const int64_t A = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kRecLanes;
    if (A >= L) return;
    const int32_t occA = leaf_start[A + 1] - leaf_start[A];
    for (int64_t e = nbr_start[A] + sub; e < nbr_start[A + 1]; e += kRecLanes) {
        const int32_t B = nbr_idx[e];
        if (rec_len) rec_len[e] = 1 + occA + leaf_start[B + 1] - leaf_start[B];
        if (tgt_len) tgt_len[e] = occA;
    }
}

// Records of leaf A, one wavefront per leaf.  The records of A's entries are
// consecutive, so A's part of the layout is one run of rows.  For each chunk
// of 64 entries the lanes load the entries' source leaves and image codes at
// once, form the record starts by a wave prefix of the record lengths
// (1 + occ_A + occ_B) and mark an LDS map from row to entry; every output row
// then finds its entry through the map (or by a forward walk over the
// starts when the chunk has more than kRecMapRows rows) and is the record's
// header, a row of A, or a row of B placed at x + s (s the entry's image),
// eight rows per lane loaded before any store.  Lanes past the end repeat the
// last row onto itself, so no load or store is conditional.
constexpr int kRecMapRows = 4096;
constexpr int kRecRows = 8;

template <bool MIXED, bool NT>
__global__ __launch_bounds__(256) void k_copy_records(
    const Row4d *__restrict__ sorted, const uint64_t *__restrict__ leaf_key,
    const int8_t *__restrict__ leaf_level, const int32_t *__restrict__ leaf_start,
    const int64_t *__restrict__ nbr_start, const int32_t *__restrict__ nbr_idx,
    const int8_t *__restrict__ nbr_shift, const int64_t *__restrict__ rec_start, int64_t L,
    Row4d *__restrict__ d8, float4 *__restrict__ d4) {
    __shared__ int32_t s_pre[4][64];     // record starts within the chunk, in rows
    __shared__ int32_t s_b0[4][64];      // first sorted slot of B
    __shared__ int32_t s_occB[4][64];
    __shared__ int32_t s_B[4][64];
    __shared__ int32_t s_code[4][64];
    __shared__ uint8_t s_map[4][kRecMapRows];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t A = p2pd::xcd_contiguous(blockIdx.x, gridDim.x) * 4 + w;
    if (A >= L) return;
    const int32_t a0 = leaf_start[A], occA = leaf_start[A + 1] - a0;
    double c[3] = {0.0, 0.0, 0.0};
    if (MIXED) {
        const uint64_t k = leaf_key[A];
        const double half = 0.5 * static_cast<double>(1u << (20 - leaf_level[A]));
        c[0] = (static_cast<double>(p2pd::compact3(k)) + half) * 0x1p-20;
        c[1] = (static_cast<double>(p2pd::compact3(k >> 1)) + half) * 0x1p-20;
        c[2] = (static_cast<double>(p2pd::compact3(k >> 2)) + half) * 0x1p-20;
    }
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
    for (int64_t c0 = e0; c0 < e1; c0 += 64) {
        const int nc = static_cast<int>(min<int64_t>(64, e1 - c0));
        int32_t len = 0, B = 0, b0 = 0, occB = 0, code = 13;
        if (lane < nc) {
            B = nbr_idx[c0 + lane];
            b0 = leaf_start[B];
            occB = leaf_start[B + 1] - b0;
            if (nbr_shift) code = nbr_shift[c0 + lane];
            len = 1 + occA + occB;
        }
        int32_t inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        s_pre[w][lane] = inc - len;
        s_b0[w][lane] = b0;
        s_occB[w][lane] = occB;
        s_B[w][lane] = B;
        s_code[w][lane] = code;
        const int32_t rows = __shfl(inc, 63, 64);
        const bool use_map = rows <= kRecMapRows;
        if (use_map)
            for (int32_t r = inc - len; r < inc; ++r) s_map[w][r] = static_cast<uint8_t>(lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int64_t d = rec_start[c0];
        int b = 0;
        for (int32_t p0 = 0; p0 < rows; p0 += 64 * kRecRows) {
            Row4d v[kRecRows];
            int32_t jq[kRecRows], rq[kRecRows];
#pragma unroll
            for (int u = 0; u < kRecRows; ++u) {
                const int32_t q = min(p0 + 64 * u + lane, rows - 1);
                int j;
                if (use_map) {
                    j = s_map[w][q];
                } else {
                    while (b + 1 < nc && s_pre[w][b + 1] <= q) ++b;
                    j = b;
                }
                const int32_t r = q - s_pre[w][j];    // 0: header, 1..occA: A's rows, then B's
                jq[u] = j;
                rq[u] = r;
                const int32_t slot = r <= occA ? a0 + max(r - 1, 0) : s_b0[w][j] + (r - 1 - occA);
                v[u] = sorted[slot];
            }
#pragma unroll
            for (int u = 0; u < kRecRows; ++u) {
                const int32_t q = min(p0 + 64 * u + lane, rows - 1);
                const int j = jq[u], r = rq[u];
                const int64_t o = d + q;
                if (r > occA) {     // a source row at its image
                    const int cd = s_code[w][j];
                    v[u].x += static_cast<double>(cd % 3 - 1);
                    v[u].y += static_cast<double>((cd / 3) % 3 - 1);
                    v[u].z += static_cast<double>(cd / 9 - 1);
                }
                if constexpr (MIXED) {
                    const float4 row = make_float4(static_cast<float>(v[u].x - c[0]), static_cast<float>(v[u].y - c[1]),
                                                   static_cast<float>(v[u].z - c[2]), static_cast<float>(v[u].w));
                    const float4 hdr = make_float4(__int_as_float(occA), __int_as_float(s_occB[w][j]),
                                                   __int_as_float(static_cast<int32_t>(A)), __int_as_float(s_B[w][j]));
                    put<NT>(d4 + o, r == 0 ? hdr : row);
                } else {
                    const Row4d hdr{static_cast<double>(occA), static_cast<double>(s_occB[w][j]),
                                    static_cast<double>(A), static_cast<double>(s_B[w][j])};
                    put<NT>(d8 + o, r == 0 ? hdr : v[u]);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

constexpr int kEvalWaves = 4;
constexpr int kRecPerWave = 8;   // consecutive records per wavefront (at most 64: one lane each)
constexpr int kRecFlush = 32;

// A wavefront takes kRecPerWave consecutive records.  Its lanes first load
// the starts, headers and result offsets of all of them at once, so that each
// record then waits for one memory round trip (its rows), not three in a
// chain.  A record's sources are staged through LDS 64 rows at a time with one
// coalesced load per lane (a load per pair straight from the record left
// every wave waiting out a memory round trip per pair group).  Targets in
// chunks of 64; with tc targets in a chunk, lane (t, g) = (lane % tc,
// lane / tc) takes target t and staged sources g, g + G, ... (G = 64 / tc),
// FP32-mixed pair terms summed at most 32 at a time in float into double;
// the G partials meet in LDS.  Record (A, A) holds every target once as its
// own source at d = 0, source row tc0 + t of target t: FP64 drops that pair
// by position, FP32-mixed adds its term back, as in the box kernels.
// With image codes only the unshifted record (A, A) is the self record: a
// point meets its own image elsewhere at a nonzero distance.
template <bool MIXED, bool EPS0>
__global__ __launch_bounds__(64 * kEvalWaves) void k_eval_records(
    const int64_t *__restrict__ rec_start, const Row4d *__restrict__ r8, const float4 *__restrict__ r4,
    const int8_t *__restrict__ nbr_shift, int64_t E, const int64_t *__restrict__ res_start, double eps2,
    Row4d *__restrict__ res) {
    using Src = typename std::conditional<MIXED, float4, Row4d>::type;
    __shared__ double s_red[kEvalWaves][4][64];
    __shared__ Src s_src[kEvalWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t eb = (static_cast<int64_t>(blockIdx.x) * kEvalWaves + w) * kRecPerWave;
    if (eb >= E) return;
    const int nrec = static_cast<int>(min<int64_t>(kRecPerWave, E - eb));
    // lane k < nrec: record eb + k
    int64_t my_r = 0, my_out = 0;
    int my_occA = 0, my_occB = 0, my_self = 0;
    if (lane < nrec) {
        const int64_t e = eb + lane;
        my_r = rec_start[e];
        my_out = res_start[e];
        int A, B;
        if constexpr (MIXED) {
            const float4 h = r4[my_r];
            my_occA = __float_as_int(h.x);
            my_occB = __float_as_int(h.y);
            A = __float_as_int(h.z);
            B = __float_as_int(h.w);
        } else {
            const Row4d h = r8[my_r];
            my_occA = static_cast<int>(h.x);
            my_occB = static_cast<int>(h.y);
            A = static_cast<int>(h.z);
            B = static_cast<int>(h.w);
        }
        my_self = (A == B && (nbr_shift == nullptr || nbr_shift[e] == 13)) ? 1 : 0;
    }
    const float eps2f = static_cast<float>(eps2);
    for (int k = 0; k < nrec; ++k) {
        const int64_t r = static_cast<int64_t>(__shfl(static_cast<long long>(my_r), k, 64));
        const int64_t out0 = static_cast<int64_t>(__shfl(static_cast<long long>(my_out), k, 64));
        const int occA = __builtin_amdgcn_readfirstlane(__shfl(my_occA, k, 64));
        const int occB = __builtin_amdgcn_readfirstlane(__shfl(my_occB, k, 64));
        const bool self = __builtin_amdgcn_readfirstlane(__shfl(my_self, k, 64)) != 0;
        const int64_t t0 = r + 1, s0 = r + 1 + occA;
        for (int tc0 = 0; tc0 < occA; tc0 += 64) {
            const int tc = min(64, occA - tc0);
            const int G = 64 / tc;
            const int t = lane % tc, g = lane / tc;
            const bool active = g < G;
            double p = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
            double tm = 0.0;
            Src tv;
            if constexpr (MIXED)
                tv = r4[t0 + tc0 + t];
            else
                tv = r8[t0 + tc0 + t];
            tm = tv.w;
            for (int b0 = 0; b0 < occB; b0 += 64) {
                const int nb = min(64, occB - b0);
                if (lane < nb) {
                    if constexpr (MIXED)
                        s_src[w][lane] = r4[s0 + b0 + lane];
                    else
                        s_src[w][lane] = r8[s0 + b0 + lane];
                }
                wave_sync();
                if (active) {
                    if constexpr (MIXED) {
                        int j = g;
                        while (j < nb) {
                            float pf = 0.f, xf = 0.f, yf = 0.f, zf = 0.f;
                            for (int k = 0; k < kRecFlush && j < nb; ++k, j += G) {
                                const float4 v = s_src[w][j];
                                const float dx = tv.x - v.x, dy = tv.y - v.y, dz = tv.z - v.z;
                                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
                                float wv = rsq_f32(r2);
                                if constexpr (EPS0) wv = (r2 > 0.f) ? wv : 0.f;
                                const float mw = v.w * wv;
                                const float mw3 = mw * (wv * wv);
                                pf -= mw;
                                xf = fmaf(-mw3, dx, xf);
                                yf = fmaf(-mw3, dy, yf);
                                zf = fmaf(-mw3, dz, zf);
                            }
                            p += pf;
                            fx += xf;
                            fy += yf;
                            fz += zf;
                        }
                    } else {
                        // the chunk step of the target's own row in the self record, else -1
                        const int selfj = (!EPS0 && self) ? tc0 + t - b0 : -1;
                        for (int j = g; j < nb; j += G) {
                            const Row4d v = s_src[w][j];
                            const double dx = tv.x - v.x, dy = tv.y - v.y, dz = tv.z - v.z;
                            const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                            double wv = p2pd::rsqrt_normal(r2);
                            if constexpr (EPS0) wv = (r2 > 0.0) ? wv : 0.0;
                            wv = (j == selfj) ? 0.0 : wv;
                            const double mw = v.w * wv;
                            const double mw3 = mw * (wv * wv);
                            p -= mw;
                            fx = fma(-mw3, dx, fx);
                            fy = fma(-mw3, dy, fy);
                            fz = fma(-mw3, dz, fz);
                        }
                    }
                }
                wave_sync();   // every lane has read this chunk before the next overwrites it
            }
            if (!active) p = fx = fy = fz = 0.0;
            s_red[w][0][lane] = p;
            s_red[w][1][lane] = fx;
            s_red[w][2][lane] = fy;
            s_red[w][3][lane] = fz;
            wave_sync();
            if (lane < tc) {
                double sp = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
                for (int q = 0; q < G; ++q) {
                    sp += s_red[w][0][q * tc + lane];
                    sx += s_red[w][1][q * tc + lane];
                    sy += s_red[w][2][q * tc + lane];
                    sz += s_red[w][3][q * tc + lane];
                }
                if (MIXED && !EPS0 && self) sp += static_cast<double>(static_cast<float>(tm) * rsq_f32(eps2f));
                res[out0 + tc0 + lane] = Row4d{sp, sx, sy, sz};
            }
            wave_sync();
        }
    }
}

// Update: for every target of leaf A, the sum of its result rows over the
// records of nbr(A), in list order, written to caller order (wave per leaf).
__global__ __launch_bounds__(256) void k_reduce_records(const int32_t *__restrict__ leaf_start,
                                                        const int64_t *__restrict__ nbr_start,
                                                        const int64_t *__restrict__ res_start,
                                                        const int32_t *__restrict__ perm, int64_t L,
                                                        const Row4d *__restrict__ res,
                                                        double *__restrict__ phi, double *__restrict__ ax,
                                                        double *__restrict__ ay, double *__restrict__ az) {
    // the result offsets of up to 64 records, staged once per chunk so that
    // the row loads do not each wait for their offset first
    __shared__ int64_t s_off[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t A = static_cast<int64_t>(blockIdx.x) * 4 + w;
    if (A >= L) return;
    const int32_t a0 = leaf_start[A], occA = leaf_start[A + 1] - a0;
    const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
    for (int t0 = 0; t0 < occA; t0 += 64) {
        const int t = t0 + lane;
        const bool act = t < occA;
        double sp = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t c0 = e0; c0 < e1; c0 += 64) {
            const int nc = static_cast<int>(min<int64_t>(64, e1 - c0));
            if (lane < nc) s_off[w][lane] = res_start[c0 + lane];
            wave_sync();
            if (act) {
                // four rows in flight, added in list order
                int k = 0;
                for (; k + 4 <= nc; k += 4) {
                    const Row4d v0 = res[s_off[w][k] + t], v1 = res[s_off[w][k + 1] + t];
                    const Row4d v2 = res[s_off[w][k + 2] + t], v3 = res[s_off[w][k + 3] + t];
                    sp += v0.x; sx += v0.y; sy += v0.z; sz += v0.w;
                    sp += v1.x; sx += v1.y; sy += v1.z; sz += v1.w;
                    sp += v2.x; sx += v2.y; sy += v2.z; sz += v2.w;
                    sp += v3.x; sx += v3.y; sy += v3.z; sz += v3.w;
                }
                for (; k < nc; ++k) {
                    const Row4d v = res[s_off[w][k] + t];
                    sp += v.x; sx += v.y; sy += v.z; sz += v.w;
                }
            }
            wave_sync();   // every lane has read the offsets before the next chunk overwrites them
        }
        if (act) {
            const int64_t i = perm[a0 + t];
            phi[i] = sp;
            ax[i] = sx;
            ay[i] = sy;
            az[i] = sz;
        }
    }
}

}  // namespace

p2p_status launch_record_lengths(const int32_t *leaf_start, const int64_t *nbr_start,
                                 const int32_t *nbr_idx, int64_t L, int32_t *rec_len, int32_t *tgt_len,
                                 hipStream_t s) {
    if (L <= 0) return P2P_OK;
    k_record_lengths<<<grid_for(L * kRecLanes, 256), 256, 0, s>>>(leaf_start, nbr_start, nbr_idx, L,
                                                                  rec_len, tgt_len);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_copy_records(const Row4d *sorted, const uint64_t *leaf_key, const int8_t *leaf_level,
                               const int32_t *leaf_start, const int64_t *nbr_start,
                               const int32_t *nbr_idx, const int8_t *nbr_shift, const int64_t *rec_start,
                               int64_t L, Row4d *d8, float4 *d4, bool streaming, hipStream_t s) {
    if (L <= 0) return P2P_OK;
    const unsigned g = grid_for(L, 4);
#define P2P_REC(M, NT)                                                                                \
    k_copy_records<M, NT><<<g, 256, 0, s>>>(sorted, leaf_key, leaf_level, leaf_start, nbr_start, nbr_idx, \
                                            nbr_shift, rec_start, L, d8, d4)
    if (d4) {
        if (streaming) P2P_REC(true, true); else P2P_REC(true, false);
    } else {
        if (streaming) P2P_REC(false, true); else P2P_REC(false, false);
    }
#undef P2P_REC
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_eval_records(const int64_t *rec_start, const Row4d *r8, const float4 *r4,
                               const int8_t *nbr_shift, int64_t E, const int64_t *res_start, double eps2,
                               bool eps_zero, Row4d *res, hipStream_t s) {
    if (E <= 0) return P2P_OK;
    const unsigned g = grid_for((E + kRecPerWave - 1) / kRecPerWave, kEvalWaves);
    const unsigned b = 64 * kEvalWaves;
#define P2P_EVAL_REC(M, E0) \
    k_eval_records<M, E0><<<g, b, 0, s>>>(rec_start, r8, r4, nbr_shift, E, res_start, eps2, res)
    if (r4) {
        if (eps_zero) P2P_EVAL_REC(true, true); else P2P_EVAL_REC(true, false);
    } else {
        if (eps_zero) P2P_EVAL_REC(false, true); else P2P_EVAL_REC(false, false);
    }
#undef P2P_EVAL_REC
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_reduce_records(const int32_t *leaf_start, const int64_t *nbr_start,
                                 const int64_t *res_start, const int32_t *perm, int64_t L,
                                 const Row4d *res, double *phi, double *ax, double *ay, double *az,
                                 hipStream_t s) {
    if (L <= 0) return P2P_OK;
    k_reduce_records<<<grid_for(L, 4), 256, 0, s>>>(leaf_start, nbr_start, res_start, perm, L, res, phi, ax,
                                                    ay, az);
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace p2p
