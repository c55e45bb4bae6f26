// Near-field gravity (gather and redundant layouts, Sec. 5.2.1, with the
// update fused; FP64 or FP32-mixed) and its adjoint.
//
// One 256-thread workgroup owns one target leaf.  Leaves hold 1..64 targets
// in an adaptive tree, so lanes are split two ways: with tc targets in the
// current chunk, lane (t, g) = (tid % tc, tid / tc) takes target t and the
// g-th of G = 256 / tc contiguous runs of every source tile, and the G
// partial sums of a target are reduced through LDS at the end.  Sources are staged
// through LDS in tiles of 512:
//   - redundant: one contiguous segment, read with coalesced loads;
//   - gather: the near list is walked in chunks; each staged row is located
//     by a binary search over the prefix of neighbour occupancies.
// Results are written straight to caller order through perm (the update
// step).  No atomics: each output has one owner.
//
// Self pair: the near field holds the target itself exactly once, at d = 0.
// FP64 drops it by position: the workgroup knows where its own leaf's rows
// sit among the staged sources, so each lane knows the one step of its run
// that is its target's own row and gives that pair weight zero (a compare
// and a select per pair, and the sums hold only the pairs of the
// definition).  FP32_MIXED saves those two slots of its fifteen: it sums over
// all sources and afterwards adds back the self term of phi (m_i
// (eps^2)^{-1/2}, computed in the same arithmetic; the self term of a is
// exactly zero), which leaves the rounding of the float partial that held
// -m_i/eps in phi_i (bounded by the smallest eps the entry points accept).
// With eps == 0 pairs at zero distance contribute nothing instead.
//
// Remote lists (sources of another particle set, REMOTE): most target leaves
// of a domain have no remote source and leave at once; the others read their
// targets and (gather) their sources through the trees' permutations straight
// from the caller-order arrays, since only a thin layer at the domain's faces
// takes part; the redundant layout reads the remote segments.  No self pair is
// added back, and the sums are added to the outputs.
//
// Periodic lists (gather and adjoint): a staged source row of an entry with
// image code c is shifted by (sx, sy, sz) domain edges, x + s in double, before
// the conversion; the redundant layout already holds shifted rows.
//
// FP32_MIXED: coordinates are taken relative to the centre of the target leaf
// in double and rounded to float once per (target leaf, source) -- the
// redundant layout stores them that way, the gather layout converts while
// staging -- so the large offset is removed in double and every pair
// difference is a float difference of small numbers; the rest of the pair
// arithmetic is float; each lane sums at most 32 pair terms in float before
// adding them to double accumulators.  Sources sit in LDS as float4 (x, y, z,
// m) for FP32_MIXED and double4 for FP64, and the source loop is unrolled by
// four with a trip count shared by all lanes.
#include <type_traits>

#include "p2p_internal.h"

namespace p2p {
namespace {

constexpr int kGBlock = 256;
constexpr int kGTile = 512;
constexpr int kGNbrChunk = 256;
constexpr int kGFlush = 32;

// Block-wide: loads one chunk of the near list of A into LDS (first sorted
// slot of each neighbour, exclusive prefix of their occupancies and, with
// PER, the image codes).
// *s_self: the first chunk row of the entry (A, unshifted), the target leaf's
// own rows, or -1 when the chunk does not hold it.
template <bool PER>
__device__ int64_t g_load_nbr_chunk(const int32_t *__restrict__ leaf_start,
                                    const int32_t *__restrict__ nbr_idx,
                                    const int8_t *__restrict__ nbr_shift, int64_t A, int64_t c0, int nc,
                                    int64_t *s_pre, int32_t *s_first, int8_t *s_code, int64_t *s_w,
                                    int64_t *s_self) {
    int32_t occ = 0, first = 0;
    bool self = false;
    if (threadIdx.x == 0) *s_self = -1;
    if (static_cast<int>(threadIdx.x) < nc) {
        const int32_t B = nbr_idx[c0 + threadIdx.x];
        first = leaf_start[B];
        occ = leaf_start[B + 1] - first;
        int code = 13;
        if constexpr (PER) {
            code = nbr_shift[c0 + threadIdx.x];
            s_code[threadIdx.x] = static_cast<int8_t>(code);
        }
        self = B == A && code == 13;
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
#pragma unroll
    for (int q = 0; q < kGBlock / 64; ++q) {
        if (q < w) woff += s_w[q];
        tot += s_w[q];
    }
    s_pre[threadIdx.x] = woff + x - occ;
    if (self) *s_self = woff + x - occ;
    if (threadIdx.x == 0) s_pre[nc] = tot;
    __syncthreads();
    return tot;
}

__device__ inline int g_find_nbr(const int64_t *s_pre, int nc, int64_t p) {
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Tile position given to `body` when the tile holds none of the target
// leaf's own rows.
constexpr int64_t kNoSelf = -(int64_t(1) << 40);

// Walks the sources of leaf A tile by tile: after a barrier, `begin(n_tile)`,
// then `stage(i, src_row, image_code)` for the tile's sources i (code 13
// unless PER), a barrier, and `body(n_tile, self)`, where tile position
// self + r holds row r of A's own rows (the unshifted entry A of its list;
// kNoSelf where no tile position does; the redundant layout takes it from
// red_self, or none if red_self is null).  Must be called by the whole block.
template <bool RED, bool PER, class Begin, class Stage, class Body>
__device__ void for_each_source_tile(int64_t A, const int64_t *__restrict__ red_start,
                                     const int32_t *__restrict__ red_self,
                                     const int64_t *__restrict__ nbr_start,
                                     const int32_t *__restrict__ nbr_idx,
                                     const int8_t *__restrict__ nbr_shift,
                                     const int32_t *__restrict__ leaf_start, int64_t *s_pre,
                                     int32_t *s_first, int8_t *s_code, int64_t *s_w, int64_t *s_self,
                                     Begin begin, Stage stage, Body body) {
    if constexpr (RED) {
        const int64_t seg0 = red_start[A], ns = red_start[A + 1] - seg0;
        const int64_t self = red_self ? static_cast<int64_t>(red_self[A]) : int64_t(-1);
        for (int64_t s0 = 0; s0 < ns; s0 += kGTile) {
            const int nt = static_cast<int>(min<int64_t>(kGTile, ns - s0));
            __syncthreads();
            begin(nt);
            for (int i = threadIdx.x; i < nt; i += kGBlock) stage(i, seg0 + s0 + i, 13);
            __syncthreads();
            body(nt, self >= 0 ? self - s0 : kNoSelf);
        }
    } else {
        const int64_t e0 = nbr_start[A], e1 = nbr_start[A + 1];
        for (int64_t c0 = e0; c0 < e1; c0 += kGNbrChunk) {
            const int nc = static_cast<int>(min<int64_t>(kGNbrChunk, e1 - c0));
            __syncthreads();
            const int64_t rows = g_load_nbr_chunk<PER>(leaf_start, nbr_idx, nbr_shift, A, c0, nc, s_pre, s_first,
                                                       s_code, s_w, s_self);
            const int64_t self = *s_self;
            for (int64_t s0 = 0; s0 < rows; s0 += kGTile) {
                const int nt = static_cast<int>(min<int64_t>(kGTile, rows - s0));
                __syncthreads();
                begin(nt);
                for (int i = threadIdx.x; i < nt; i += kGBlock) {
                    const int64_t p = s0 + i;
                    const int b = g_find_nbr(s_pre, nc, p);
                    stage(i, s_first[b] + (p - s_pre[b]), PER ? static_cast<int>(s_code[b]) : 13);
                }
                __syncthreads();
                body(nt, self >= 0 ? self - s0 : kNoSelf);
            }
        }
    }
}

// Source row of an entry with image code c, placed at x + s in double.
__device__ inline Row4d shifted(Row4d v, int c) {
    v.x += static_cast<double>(c % 3 - 1);
    v.y += static_cast<double>((c / 3) % 3 - 1);
    v.z += static_cast<double>(c / 9 - 1);
    return v;
}

__device__ inline float rsq_f32(float x) { return __builtin_amdgcn_rsqf(x); }

// Lane split of a workgroup for tc targets (1 <= tc <= 256): G = 256 / tc
// groups, lane tid = t + g tc, without integer division.  For 0 <= v <= 256,
// (v + 1/2) / tc lies at least 1/(2 tc) from an integer, far beyond the error
// of the approximate reciprocal and one rounding (under 5e-5 / tc), so
// truncation gives floor(v / tc) exactly.
__device__ inline void lane_split(int tc, int &G, int &t, int &g) {
    const float rtc = __builtin_amdgcn_rcpf(static_cast<float>(tc));
    G = static_cast<int>((static_cast<float>(kGBlock) + 0.5f) * rtc);
    g = static_cast<int>((static_cast<float>(threadIdx.x) + 0.5f) * rtc);
    t = static_cast<int>(threadIdx.x) - g * tc;
}

// Centre of a particle leaf (exact in double: integers below 2^21 times 2^-20).
__device__ inline void leaf_centre(uint64_t key, int level, double c[3]) {
    const double half = 0.5 * static_cast<double>(1u << (20 - level));
    c[0] = (static_cast<double>(p2pd::compact3(key)) + half) * 0x1p-20;
    c[1] = (static_cast<double>(p2pd::compact3(key >> 1)) + half) * 0x1p-20;
    c[2] = (static_cast<double>(p2pd::compact3(key >> 2)) + half) * 0x1p-20;
}

// Source row at sorted slot `row` of the gather layout: the sorted rows, or for
// remote sources the caller-order arrays through the source tree's perm.
template <bool REMOTE>
__device__ inline Row4d source_row(const GravityArgs &a, int64_t row) {
    if constexpr (REMOTE) {
        const int64_t j = a.src_perm[row];
        return Row4d{a.sx[j], a.sy[j], a.sz[j], a.sm[j]};
    } else {
        return a.s4[row];
    }
}

template <bool MIXED, bool RED, bool EPS0, bool PER, bool REMOTE>
__device__ __forceinline__ void gravity_body(const GravityArgs &a) {
    using Src = typename std::conditional<MIXED, float4, Row4d>::type;
    // a tile of kGTile sources padded to G equal runs (see below): at most
    // kGTile + kGBlock - 1 entries; the per-target reduction reuses the same
    // memory after the last tile
    __shared__ Src s_src[kGTile + kGBlock];
    __shared__ int64_t s_pre[kGNbrChunk + 1];
    __shared__ int32_t s_first[kGNbrChunk];
    __shared__ int8_t s_code[PER ? kGNbrChunk : 1];
    __shared__ int64_t s_w[kGBlock / 64];
    __shared__ int64_t s_self;
    static_assert(sizeof(s_src) >= 4 * kGBlock * sizeof(double), "reduction does not fit");
    double(*s_red)[kGBlock] = reinterpret_cast<double(*)[kGBlock]>(s_src);
    // FP64 with eps > 0 drops the target's own pair by position (see the top)
    constexpr bool MASK = !MIXED && !EPS0 && !REMOTE;

    // gather: neighbouring leaves on one XCD share their sources in its L2
    const int64_t A = RED ? static_cast<int64_t>(blockIdx.x) : p2pd::xcd_contiguous(blockIdx.x, gridDim.x);
    if constexpr (REMOTE) {
        if (a.nbr_start[A] == a.nbr_start[A + 1]) return;   // the whole workgroup: no barrier is skipped
    }
    const int32_t t0 = a.leaf_start[A];
    const int32_t ntar = a.leaf_start[A + 1] - t0;
    const double eps2 = a.eps2;
    const float eps2f = static_cast<float>(a.eps2);
    double c[3] = {0.0, 0.0, 0.0};
    if (MIXED) leaf_centre(a.leaf_key[A], a.leaf_level[A], c);

    for (int tc0 = 0; tc0 < ntar; tc0 += kGBlock) {
        const int tc = min(kGBlock, ntar - tc0);
        int G, t, g;
        lane_split(tc, G, t, g);
        const bool active = g < G;
        // target position (relative to the leaf centre for FP32_MIXED) and mass
        Src tv;
        if constexpr (REMOTE) {
            const int64_t i = a.perm[t0 + tc0 + t];
            const Row4d v{a.tx[i], a.ty[i], a.tz[i], 0.0};
            if constexpr (MIXED)
                tv = make_float4(static_cast<float>(v.x - c[0]), static_cast<float>(v.y - c[1]),
                                 static_cast<float>(v.z - c[2]), static_cast<float>(v.w));
            else
                tv = v;
        } else if constexpr (MIXED) {
            if constexpr (RED) {
                tv = a.red4[a.red_start[A] + a.red_self[A] + tc0 + t];
            } else {
                const Row4d v = a.s4[t0 + tc0 + t];
                tv = make_float4(static_cast<float>(v.x - c[0]), static_cast<float>(v.y - c[1]),
                                 static_cast<float>(v.z - c[2]), static_cast<float>(v.w));
            }
        } else {
            tv = a.s4[RED ? a.red_start[A] + a.red_self[A] + tc0 + t : t0 + tc0 + t];
        }
        double p = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;

        // Tile layout: lane group g takes the contiguous run of sources
        // [g chunk, (g + 1) chunk) of the tile, chunk = ceil(nt / G).  The
        // G chunk - nt entries past the end are zero-mass sources far away
        // (they add exact zeros), so every lane runs the same trip count and
        // the four reads of an unrolled step sit at fixed offsets from one
        // address.
        int chunk = 0;
        auto begin = [&](int nt) {
            chunk = (nt + G - 1) / G;
            for (int i = nt + static_cast<int>(threadIdx.x); i < G * chunk; i += kGBlock) {
                if constexpr (MIXED)
                    s_src[i] = make_float4(1e18f, 1e18f, 1e18f, 0.f);
                else
                    s_src[i] = Row4d{1e18, 1e18, 1e18, 0.0};
            }
        };
        auto stage = [&](int i, int64_t row, int code) {
            Src *d = s_src + i;
            if constexpr (MIXED) {
                if constexpr (RED) {
                    *d = a.red4[row];
                } else {
                    Row4d v = source_row<REMOTE>(a, row);
                    if constexpr (PER) v = shifted(v, code);
                    *d = make_float4(static_cast<float>(v.x - c[0]), static_cast<float>(v.y - c[1]),
                                     static_cast<float>(v.z - c[2]), static_cast<float>(v.w));
                }
            } else {
                if constexpr (RED)
                    *d = a.s4[row];
                else if constexpr (PER)
                    *d = shifted(source_row<REMOTE>(a, row), code);
                else
                    *d = source_row<REMOTE>(a, row);
            }
        };
        auto body = [&](int nt, int64_t self) {
            if (!active) return;
            const Src *sp = s_src + g * chunk;
            // MASK: the step of this lane's run at its target's own row, else -1
            int selfj = -1;
            if constexpr (MASK) {
                const int64_t pos = self + tc0 + t;
                const int64_t j = pos - static_cast<int64_t>(g) * chunk;
                if (pos >= 0 && pos < nt && j >= 0 && j < chunk) selfj = static_cast<int>(j);
            }
            if constexpr (MIXED) {
                auto pair = [&](const float4 v, float &pf, float &xf, float &yf, float &zf) {
                    const float dx = tv.x - v.x, dy = tv.y - v.y, dz = tv.z - v.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
                    float w = rsq_f32(r2);
                    if constexpr (EPS0) w = (r2 > 0.f) ? w : 0.f;
                    const float mw = v.w * w;
                    const float mw3 = mw * (w * w);
                    pf -= mw;
                    xf = fmaf(-mw3, dx, xf);
                    yf = fmaf(-mw3, dy, yf);
                    zf = fmaf(-mw3, dz, zf);
                };
                for (int k0 = 0; k0 < chunk; k0 += kGFlush) {
                    const int kk = min(kGFlush, chunk - k0);
                    float pf = 0.f, xf = 0.f, yf = 0.f, zf = 0.f;
                    int j = 0;
                    for (; j + 4 <= kk; j += 4, sp += 4) {
                        const float4 v0 = sp[0], v1 = sp[1], v2 = sp[2], v3 = sp[3];
                        pair(v0, pf, xf, yf, zf);
                        pair(v1, pf, xf, yf, zf);
                        pair(v2, pf, xf, yf, zf);
                        pair(v3, pf, xf, yf, zf);
                    }
                    for (; j < kk; ++j, ++sp) pair(sp[0], pf, xf, yf, zf);
                    p += pf;
                    fx += xf;
                    fy += yf;
                    fz += zf;
                }
            } else {
                auto pair = [&](const Row4d v, int j) {
                    const double dx = tv.x - v.x, dy = tv.y - v.y, dz = tv.z - v.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                    double w = p2pd::rsqrt_normal(r2);
                    if constexpr (EPS0) w = (r2 > 0.0) ? w : 0.0;
                    if constexpr (MASK) w = (j == selfj) ? 0.0 : w;
                    const double mw = v.w * w;
                    const double mw3 = mw * (w * w);
                    p -= mw;
                    fx = fma(-mw3, dx, fx);
                    fy = fma(-mw3, dy, fy);
                    fz = fma(-mw3, dz, fz);
                };
                int j = 0;
                for (; j + 4 <= chunk; j += 4, sp += 4) {
                    const Row4d v0 = sp[0], v1 = sp[1], v2 = sp[2], v3 = sp[3];
                    pair(v0, j);
                    pair(v1, j + 1);
                    pair(v2, j + 2);
                    pair(v3, j + 3);
                }
                for (; j < chunk; ++j, ++sp) pair(sp[0], j);
            }
        };
        for_each_source_tile<RED, PER>(A, a.red_start, REMOTE ? nullptr : a.red_self, a.nbr_start, a.nbr_idx,
                                       a.nbr_shift, a.src_leaf_start, s_pre, s_first, s_code, s_w, &s_self,
                                       begin, stage, body);

        // Per-target sums of the G partials, in the order q = 0..G-1.  Lanes
        // with g >= G never accumulate and are never read.  When 4 tc <= 256,
        // lane (t, g) with g < 4 sums component g of target t (it already
        // holds target t's row), so the four sums of a target run in four
        // lanes; otherwise lane t sums all four.
        __syncthreads();
        s_red[0][threadIdx.x] = p;
        s_red[1][threadIdx.x] = fx;
        s_red[2][threadIdx.x] = fy;
        s_red[3][threadIdx.x] = fz;
        __syncthreads();
        // FP32_MIXED: the self pair (d = 0) of phi, computed in the same arithmetic
        auto self_phi = [&]() -> double {
            if constexpr (MIXED)
                return static_cast<double>(tv.w * rsq_f32(eps2f));
            else
                return tv.w * rsqrt(eps2);
        };
        if (4 * tc <= kGBlock) {
            if (g < 4) {
                double s = 0.0;
                for (int q = 0; q < G; ++q) s += s_red[g][q * tc + t];
                if constexpr (MIXED && !EPS0 && !REMOTE) {
                    if (g == 0) s += self_phi();
                }
                double *out = g == 0 ? a.phi : g == 1 ? a.ax : g == 2 ? a.ay : a.az;
                const int64_t i = a.perm[t0 + tc0 + t];
                if constexpr (REMOTE)
                    out[i] += s;
                else
                    out[i] = s;
            }
        } else if (static_cast<int>(threadIdx.x) < tc) {
            double sp_ = 0.0, sx_ = 0.0, sy_ = 0.0, sz_ = 0.0;
            for (int q = 0; q < G; ++q) {
                const int l = q * tc + threadIdx.x;
                sp_ += s_red[0][l];
                sx_ += s_red[1][l];
                sy_ += s_red[2][l];
                sz_ += s_red[3][l];
            }
            if constexpr (MIXED && !EPS0 && !REMOTE) sp_ += self_phi();
            const int64_t i = a.perm[t0 + tc0 + threadIdx.x];
            if constexpr (REMOTE) {
                a.phi[i] += sp_;
                a.ax[i] += sx_;
                a.ay[i] += sy_;
                a.az[i] += sz_;
            } else {
                a.phi[i] = sp_;
                a.ax[i] = sx_;
                a.ay[i] = sy_;
                a.az[i] = sz_;
            }
        }
    }
}

// The FP32-mixed redundant kernel fits in 64 VGPRs without spills, so it asks
// for 8 waves per SIMD (more workgroups in flight hide the tile staging); the
// FP32-mixed gather kernel fits 72 without spills (7 waves per SIMD), its
// periodic form 80 (6 waves per SIMD; at 72 it spills); the FP64 variants keep
// the compiler's register budget.  PER: periodic gather.
template <bool MIXED, bool RED, bool EPS0, bool PER, bool REMOTE>
__global__ __launch_bounds__(kGBlock) void k_gravity(GravityArgs a) {
    gravity_body<MIXED, RED, EPS0, PER, REMOTE>(a);
}
template <bool EPS0>
__global__ __launch_bounds__(kGBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_gravity_mixed_red(
    GravityArgs a) {
    gravity_body<true, true, EPS0, false, false>(a);
}
template <bool EPS0>
__global__ __launch_bounds__(kGBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_gravity_mixed_gather(
    GravityArgs a) {
    gravity_body<true, false, EPS0, false, false>(a);
}
template <bool EPS0>
__global__ __launch_bounds__(kGBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_gravity_mixed_gather_per(
    GravityArgs a) {
    gravity_body<true, false, EPS0, true, false>(a);
}

// Adjoint of the gravity sums, gather layout.  For target j and each near
// source k (d = x_j - x_k, w = (|d|^2+eps^2)^{-1/2}):
//   g_x_j += [ m_k (gp_j w^3 + 3 w^5 ga_j.d) + m_j (gp_k w^3 - 3 w^5 ga_k.d) ] d
//            + w^3 (m_j ga_k - m_k ga_j)
//   g_m_j += -(gp_k w - w^3 ga_k.d)
// (the derivative of L = sum_i gp_i phi_i + ga_i . a_i through both the pair
// (j, k) and the pair (k, j)).  The self pair adds zero to g_x and
// -gp_j/eps to g_m: FP64 drops it by position, FP32_MIXED adds it back, as in
// the forward kernels.  FP32_MIXED as in the forward
// kernels: positions relative to the target leaf's centre, taken in double
// and rounded to float once per staged source, float pair terms summed at
// most 32 at a time before they are added to double accumulators.
// Five waves per SIMD: the FP32-mixed form then fits in 96 registers without
// spills (15% faster than at four); the FP64 form runs as fast either way.
template <bool PER, bool MIXED>
__global__ __launch_bounds__(kGBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_gravity_adjoint(
    GravityAdjointArgs a) {
    using Src = typename std::conditional<MIXED, float4, Row4d>::type;
    __shared__ Src s_p[kGTile];    // sources (x, y, z, m)
    __shared__ Src s_g[kGTile];    // their upstream gradients (g_phi, g_ax, g_ay, g_az)
    __shared__ int64_t s_pre[kGNbrChunk + 1];
    __shared__ int32_t s_first[kGNbrChunk];
    __shared__ int8_t s_code[kGNbrChunk];
    __shared__ int64_t s_w[kGBlock / 64];
    __shared__ int64_t s_self;
    static_assert(sizeof(s_g) >= 4 * kGBlock * sizeof(double), "reduction does not fit");
    double *s_red = reinterpret_cast<double *>(s_g);   // reused after the last tile

    const int64_t A = blockIdx.x;
    const int32_t t0 = a.leaf_start[A];
    const int32_t ntar = a.leaf_start[A + 1] - t0;
    const double eps2 = a.eps2;
    const float eps2f = static_cast<float>(eps2);
    double c[3] = {0.0, 0.0, 0.0};
    if (MIXED) leaf_centre(a.leaf_key[A], a.leaf_level[A], c);
    auto rel = [&](const Row4d &v) {
        return make_float4(static_cast<float>(v.x - c[0]), static_cast<float>(v.y - c[1]),
                           static_cast<float>(v.z - c[2]), static_cast<float>(v.w));
    };
    auto grad = [](const Row4d &v) {
        return make_float4(static_cast<float>(v.x), static_cast<float>(v.y), static_cast<float>(v.z),
                           static_cast<float>(v.w));
    };
    for (int tc0 = 0; tc0 < ntar; tc0 += kGBlock) {
        const int tc = min(kGBlock, ntar - tc0);
        int G, t, g;
        lane_split(tc, G, t, g);
        const bool active = g < G;
        const int64_t tr = t0 + tc0 + t;
        Src pj, gj;
        if constexpr (MIXED) {
            pj = rel(a.s4[tr]);
            gj = grad(a.g4[tr]);
        } else {
            pj = a.s4[tr];
            gj = a.g4[tr];
        }
        double om = 0.0, ox = 0.0, oy = 0.0, oz = 0.0;
        // The term w^3 (m_j ga_k - m_k ga_j) is summed as m_j sum_k w^3 ga_k -
        // ga_j sum_k w^3 m_k: two running sums instead of a difference per pair
        // (FP64 over all sources; FP32_MIXED per group of at most kGFlush pairs)
        double s1x = 0.0, s1y = 0.0, s1z = 0.0, s2 = 0.0;
        // a periodic source image at x_k + s: both pair directions see the
        // same d = x_j - (x_k + s) (the reverse entry carries -s)
        auto stage = [&](int i, int64_t row, int code) {
            const Row4d v = PER ? shifted(a.s4[row], code) : a.s4[row];
            if constexpr (MIXED) {
                s_p[i] = rel(v);
                s_g[i] = grad(a.g4[row]);
            } else {
                s_p[i] = v;
                s_g[i] = a.g4[row];
            }
        };
        auto body = [&](int nt, int64_t self) {
            if (!active) return;
            if constexpr (MIXED) {
                int s = g;
                while (s < nt) {
                    float fm = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
                    // sum w^3 ga_k and sum w^3 m_k of the group, as in FP64
                    float f1x = 0.f, f1y = 0.f, f1z = 0.f, f2 = 0.f;
                    for (int k = 0; k < kGFlush && s < nt; ++k, s += G) {
                        const float4 pk = s_p[s], gk = s_g[s];
                        const float dx = pj.x - pk.x, dy = pj.y - pk.y, dz = pj.z - pk.z;
                        const float w = rsq_f32(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f))));
                        const float w2 = w * w, w3 = w2 * w, w5 = w3 * w2;
                        const float gdj = fmaf(gj.y, dx, fmaf(gj.z, dy, gj.w * dz));
                        const float gdk = fmaf(gk.y, dx, fmaf(gk.z, dy, gk.w * dz));
                        const float cc = pk.w * fmaf(3.f * w5, gdj, gj.x * w3) + pj.w * fmaf(-3.f * w5, gdk, gk.x * w3);
                        fx = fmaf(cc, dx, fx);
                        fy = fmaf(cc, dy, fy);
                        fz = fmaf(cc, dz, fz);
                        f1x = fmaf(w3, gk.y, f1x);
                        f1y = fmaf(w3, gk.z, f1y);
                        f1z = fmaf(w3, gk.w, f1z);
                        f2 = fmaf(w3, pk.w, f2);
                        fm -= gk.x * w - w3 * gdk;
                    }
                    om += fm;
                    ox += fmaf(pj.w, f1x, fmaf(-gj.y, f2, fx));
                    oy += fmaf(pj.w, f1y, fmaf(-gj.z, f2, fy));
                    oz += fmaf(pj.w, f1z, fmaf(-gj.w, f2, fz));
                }
            } else {
                // the tile position of the target's own row, whose pair is dropped
                const int64_t pos = self + tc0 + t;
                const int selfs = (pos >= 0 && pos < nt) ? static_cast<int>(pos) : -1;
                for (int s = g; s < nt; s += G) {
                    const Row4d pk = s_p[s], gk = s_g[s];
                    const double dx = pj.x - pk.x, dy = pj.y - pk.y, dz = pj.z - pk.z;
                    double w = p2pd::rsqrt_normal(fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2))));
                    w = (s == selfs) ? 0.0 : w;
                    const double w3 = w * w * w, w5 = w3 * w * w;
                    const double gdj = gj.y * dx + gj.z * dy + gj.w * dz;
                    const double gdk = gk.y * dx + gk.z * dy + gk.w * dz;
                    const double cc = pk.w * (gj.x * w3 + 3.0 * w5 * gdj) + pj.w * (gk.x * w3 - 3.0 * w5 * gdk);
                    ox += cc * dx;
                    oy += cc * dy;
                    oz += cc * dz;
                    s1x += w3 * gk.y;
                    s1y += w3 * gk.z;
                    s1z += w3 * gk.w;
                    s2 += w3 * pk.w;
                    om -= gk.x * w - w3 * gdk;
                }
            }
        };
        for_each_source_tile<false, PER>(A, nullptr, nullptr, a.nbr_start, a.nbr_idx, a.nbr_shift, a.leaf_start,
                                         s_pre, s_first, s_code, s_w, &s_self, [](int) {}, stage, body);
        if constexpr (!MIXED) {
            ox += pj.w * s1x - gj.y * s2;
            oy += pj.w * s1y - gj.z * s2;
            oz += pj.w * s1z - gj.w * s2;
        }
        __syncthreads();
        s_red[0 * kGBlock + threadIdx.x] = active ? om : 0.0;
        s_red[1 * kGBlock + threadIdx.x] = active ? ox : 0.0;
        s_red[2 * kGBlock + threadIdx.x] = active ? oy : 0.0;
        s_red[3 * kGBlock + threadIdx.x] = active ? oz : 0.0;
        __syncthreads();
        if (static_cast<int>(threadIdx.x) < tc) {
            double r[4] = {0.0, 0.0, 0.0, 0.0};
            for (int q = 0; q < G; ++q)
                for (int cI = 0; cI < 4; ++cI) r[cI] += s_red[cI * kGBlock + q * tc + threadIdx.x];
            // FP32_MIXED: the self pair added -g_phi_j / eps to g_m, in the same arithmetic
            if constexpr (MIXED) r[0] += static_cast<double>(gj.x * rsq_f32(eps2f));
            const int64_t i = a.perm[t0 + tc0 + threadIdx.x];
            a.gm[i] = r[0];
            a.gx[i] = r[1];
            a.gy[i] = r[2];
            a.gz[i] = r[3];
        }
        __syncthreads();
    }
}

}  // namespace

p2p_status launch_gravity(const GravityArgs &a, bool redundant, bool mixed, bool eps_zero,
                          hipStream_t s) {
    if (a.L <= 0) return P2P_OK;
    const unsigned g = static_cast<unsigned>(a.L);
    // the redundant layout holds shifted rows already; only the gather stages images
    const bool per = !redundant && a.nbr_shift != nullptr;
#define P2P_GRAV(M, R, E, P) k_gravity<M, R, E, P, false><<<g, kGBlock, 0, s>>>(a)
    if (mixed) {
        if (redundant) {
            if (eps_zero) k_gravity_mixed_red<true><<<g, kGBlock, 0, s>>>(a);
            else k_gravity_mixed_red<false><<<g, kGBlock, 0, s>>>(a);
        } else if (per) {
            if (eps_zero) k_gravity_mixed_gather_per<true><<<g, kGBlock, 0, s>>>(a);
            else k_gravity_mixed_gather_per<false><<<g, kGBlock, 0, s>>>(a);
        } else {
            if (eps_zero) k_gravity_mixed_gather<true><<<g, kGBlock, 0, s>>>(a);
            else k_gravity_mixed_gather<false><<<g, kGBlock, 0, s>>>(a);
        }
    } else {
        if (redundant) {
            if (eps_zero) P2P_GRAV(false, true, true, false); else P2P_GRAV(false, true, false, false);
        } else if (per) {
            if (eps_zero) P2P_GRAV(false, false, true, true); else P2P_GRAV(false, false, false, true);
        } else {
            if (eps_zero) P2P_GRAV(false, false, true, false); else P2P_GRAV(false, false, false, false);
        }
    }
#undef P2P_GRAV
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_gravity_remote(const GravityArgs &a, bool redundant, bool mixed, bool eps_zero,
                                 hipStream_t s) {
    if (a.L <= 0) return P2P_OK;
    const unsigned g = static_cast<unsigned>(a.L);
    const bool per = !redundant && a.nbr_shift != nullptr;
#define P2P_GRAV_R(M, R, E, P) k_gravity<M, R, E, P, true><<<g, kGBlock, 0, s>>>(a)
#define P2P_GRAV_RM(M)                                                                                  \
    if (redundant) { if (eps_zero) P2P_GRAV_R(M, true, true, false); else P2P_GRAV_R(M, true, false, false); } \
    else if (per) { if (eps_zero) P2P_GRAV_R(M, false, true, true); else P2P_GRAV_R(M, false, false, true); } \
    else { if (eps_zero) P2P_GRAV_R(M, false, true, false); else P2P_GRAV_R(M, false, false, false); }
    if (mixed) { P2P_GRAV_RM(true) } else { P2P_GRAV_RM(false) }
#undef P2P_GRAV_RM
#undef P2P_GRAV_R
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

p2p_status launch_gravity_adjoint(const GravityAdjointArgs &a, bool mixed, hipStream_t s) {
    if (a.L <= 0) return P2P_OK;
    const unsigned g = static_cast<unsigned>(a.L);
    if (a.nbr_shift) {
        if (mixed) k_gravity_adjoint<true, true><<<g, kGBlock, 0, s>>>(a);
        else k_gravity_adjoint<true, false><<<g, kGBlock, 0, s>>>(a);
    } else {
        if (mixed) k_gravity_adjoint<false, true><<<g, kGBlock, 0, s>>>(a);
        else k_gravity_adjoint<false, false><<<g, kGBlock, 0, s>>>(a);
    }
    P2P_LAUNCH_CHECK();
    return P2P_OK;
}

}  // namespace p2p
