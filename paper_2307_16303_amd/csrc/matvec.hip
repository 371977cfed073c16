// HODLR3D mat-vec (Algorithm 2) and its adjoint on the device.
//
//   gather   xp = x[perm]                               (sorted order)
//   near     yn_t = sum_{s in Near(t)} K(t,s) xp_s      (leaf blocks, kernel
//            entries evaluated on the fly, sources staged through LDS)
//   stage 1  z_b = V_b^T xp_s  for every far block b    (factor stream; in the
//            adjoint U_b^T xp_t)
//   stage 2  y_t = yn_t + sum_levels sum_{b of t} U_b z_b, written straight
//            to y[perm] (in the adjoint V_b z_b summed over the blocks whose
//            source is the box)
//
// Stage 1 treats every factor column as one dot product: a sub-wave of S
// lanes (S ~ the level's box size) walks one column, so 64/S consecutive
// columns, which are consecutive in memory, are read per wave instruction.
// Stage 2 gives every row its own lane (two rows for boxes of 65..128 points):
// one workgroup per box of a chunk level (boxes of roughly 64 points), looping
// over the levels; at each level the lane streams the column slices of the
// factors of the box that contains its row.  No atomics: every output row is written by exactly one lane, and the
// summation order is fixed, so results are bitwise reproducible.
#include "h3d_internal.hpp"

namespace h3d {

namespace {

// Factor loads.  Plain loads keep the lines in L2: a column slice rarely
// starts on a 128-byte line, and the part of a line that the next slice
// needs is then still cached (with the non-temporal hint such lines were
// fetched twice).  kS2NonTemporal selects the hint for the stage-2 stream.
constexpr bool kS2NonTemporal = false;

template <int DT> struct Fac;
template <> struct Fac<H3D_F64> {
    using T = double;
    static __device__ __forceinline__ double cvt(T v) { return v; }
};
template <> struct Fac<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ double cvt(T v) { return double(v); }
};
template <> struct Fac<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ double cvt(T v) {
        return double(__uint_as_float(uint32_t(v) << 16));
    }
};
template <int DT, bool NT = false>
__device__ __forceinline__ double fac_ld(const typename Fac<DT>::T *p) {
    if constexpr (NT)
        return Fac<DT>::cvt(__builtin_nontemporal_load(p));
    else
        return Fac<DT>::cvt(*p);
}

__device__ __forceinline__ double kernel_f(int kind, double kp, double r) {
    if (r == 0.0)
        return 0.0;
    switch (kind) {
    case H3D_LAPLACE:
        return 1.0 / (4.0 * 3.14159265358979323846 * r);
    case H3D_YUKAWA:
        return exp(-kp * r) / r;
    case H3D_INV_R4: {
        double r2 = r * r;
        return 1.0 / (r2 * r2);
    }
    case H3D_COS_R:
        return cos(kp * r) / r;
    default:
        return 0.0;
    }
}

// ---------------------------------------------------------------------------
__global__ void k_gather(const void *__restrict__ x, int io_f32, int64_t ldx, int64_t n, int nrhs,
                         const int32_t *__restrict__ perm, double *__restrict__ xp) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const int64_t src = perm[p];
    for (int q = 0; q < nrhs; ++q) {
        double v = io_f32 ? double(static_cast<const float *>(x)[q * ldx + src])
                          : static_cast<const double *>(x)[q * ldx + src];
        xp[q * n + p] = v;
    }
}

// ---------------------------------------------------------------------------
// near field: one wave per leaf; lane = (row within a pass of R rows, source
// slice q of Q = 64/R); sources staged through LDS in chunks of kChunk points
constexpr int kChunk = 256;

template <int NR>
__global__ void __launch_bounds__(64)
    k_near(int L, const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ near_ptr,
           const int32_t *__restrict__ near_s, const double *__restrict__ px,
           const double *__restrict__ py, const double *__restrict__ pz, int kind, double kp,
           int nrhs, const double *__restrict__ xp, int64_t n, double *__restrict__ yn) {
    __shared__ double sx[kChunk], sy[kChunk], sz[kChunk];
    __shared__ double sv[NR][kChunk];
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t t0 = leaf_off[t];
    const int m = leaf_off[t + 1] - t0;
    if (m == 0)
        return;
    int R = 1;
    while (R < m && R < 64)
        R <<= 1;
    const int Q = 64 / R;
    const int e0 = near_ptr[t], e1 = near_ptr[t + 1];
    for (int rowb = 0; rowb < m; rowb += R) {
        const int i = rowb + (lane % R);
        const int q = lane / R;
        const bool ai = i < m;
        const int64_t gi = t0 + (ai ? i : 0);
        const double xi = px[gi], yi = py[gi], zi = pz[gi];
        for (int rb = 0; rb < nrhs; rb += NR) {
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = 0.0;
            for (int e = e0; e < e1; ++e) {
                const int32_t s = near_s[e];
                const int32_t s0 = leaf_off[s];
                const int ns = leaf_off[s + 1] - s0;
                for (int cb = 0; cb < ns; cb += kChunk) {
                    const int cn = min(kChunk, ns - cb);
                    __syncthreads();
                    for (int j = lane; j < cn; j += 64) {
                        const int64_t gj = s0 + cb + j;
                        sx[j] = px[gj];
                        sy[j] = py[gj];
                        sz[j] = pz[gj];
#pragma unroll
                        for (int c = 0; c < NR; ++c)
                            sv[c][j] = (rb + c < nrhs) ? xp[(rb + c) * n + gj] : 0.0;
                    }
                    __syncthreads();
                    if (ai) {
                        for (int j = q; j < cn; j += Q) {
                            const int64_t gj = s0 + cb + j;
                            if (gj == gi)
                                continue;
                            const double dx = xi - sx[j], dy = yi - sy[j], dz = zi - sz[j];
                            const double f = kernel_f(kind, kp, sqrt(dx * dx + dy * dy + dz * dz));
#pragma unroll
                            for (int c = 0; c < NR; ++c)
                                acc[c] += f * sv[c][j];
                        }
                    }
                }
            }
            for (int off = R; off < 64; off <<= 1)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    acc[c] += __shfl_xor(acc[c], off, 64);
            if (ai && q == 0)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (rb + c < nrhs)
                        yn[(rb + c) * n + gi] = acc[c];
        }
    }
}

// ---------------------------------------------------------------------------
// stage 1: z[col] = dot(column col of its block's factor, x segment), one
// launch per level with a shape chosen for that level's box size and rank.
//
//  wide   <S, U>: item = (block, first column); NS = 64/S columns side by side
//                 (S lanes each, rows strided by S), U such groups per pass,
//                 so each lane has U independent loads in flight; block
//                 metadata is wave-uniform.
//  packed <S, U>: item = (first block, count); one sub-wave of S lanes per
//                 block, 64/S consecutive blocks per wave, U columns per pass;
//                 the column loop runs to the wave's largest rank so the
//                 shuffles stay in uniform control flow.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

struct S1Args {
    const int2 *items;
    int64_t nitems;
    int span;
    const int64_t *blk_col0;
    const int32_t *rank;
    const int32_t *seg_len;
    const int32_t *seg_off;
    void *const *seg_ptr;
    const float *scale2;
    int nrhs;
    const double *xp;
    int64_t n;
    double *z;
    int64_t ldz;
};

template <int S, int U, int DT, int NR>
__global__ void __launch_bounds__(256) k_s1_wide(S1Args a) {
    using T = typename Fac<DT>::T;
    constexpr int NS = 64 / S;
    const int64_t w = uniform64((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
    if (w >= a.nitems)
        return;
    const int2 item = a.items[w];
    const int lane = threadIdx.x & 63;
    const int r = lane % S, sub = lane / S;
    const int b = item.x;
    const int len = a.seg_len[b];
    const int64_t off = a.seg_off[b];
    const int64_t col0 = a.blk_col0[b];
    const int k = a.rank[b];
    const T *__restrict__ p = static_cast<const T *>(a.seg_ptr[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(a.scale2[2 * b]) * double(a.scale2[2 * b + 1]);
    const int cend = min(item.y + a.span, k);
    const double *__restrict__ xp = a.xp;
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        for (int cb = item.y; cb < cend; cb += NS * U) {
            double acc[U][NR];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] = 0.0;
            for (int j = r; j < len; j += S) {
                double xv[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    xv[q] = (NR == 1 || rb + q < a.nrhs) ? xp[(rb + q) * a.n + off + j] : 0.0;
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = cb + sub + u * NS;
                    v[u] = c < cend ? fac_ld<DT>(p + int64_t(c) * len + j) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        acc[u][q] += v[u] * xv[q];
            }
#pragma unroll
            for (int o = S / 2; o > 0; o >>= 1)
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        acc[u][q] += __shfl_xor(acc[u][q], o, S);
            if (r == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = cb + sub + u * NS;
                    if (c < cend)
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < a.nrhs)
                                a.z[(rb + q) * a.ldz + col0 + c] = acc[u][q] * sc;
                }
            }
        }
    }
}

template <int S, int U, int DT, int NR>
__global__ void __launch_bounds__(256) k_s1_packed(S1Args a) {
    using T = typename Fac<DT>::T;
    const int64_t w = uniform64((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
    if (w >= a.nitems)
        return;
    const int2 item = a.items[w];
    const int lane = threadIdx.x & 63;
    const int r = lane % S, sub = lane / S;
    const bool valid = sub < item.y;
    const int b = item.x + (valid ? sub : 0);
    const int len = valid ? a.seg_len[b] : 0;
    const int64_t off = a.seg_off[b];
    const int64_t col0 = a.blk_col0[b];
    const int k = valid ? a.rank[b] : 0;
    const T *__restrict__ p = static_cast<const T *>(a.seg_ptr[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(a.scale2[2 * b]) * double(a.scale2[2 * b + 1]);
    int kmax = k;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const double *__restrict__ xp = a.xp;
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        for (int cb = 0; cb < kmax; cb += U) {
            double acc[U][NR];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] = 0.0;
            for (int j = r; j < len; j += S) {
                double xv[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    xv[q] = (NR == 1 || rb + q < a.nrhs) ? xp[(rb + q) * a.n + off + j] : 0.0;
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    v[u] = cb + u < k ? fac_ld<DT>(p + int64_t(cb + u) * len + j) : 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        acc[u][q] += v[u] * xv[q];
            }
#pragma unroll
            for (int o = S / 2; o > 0; o >>= 1)
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        acc[u][q] += __shfl_xor(acc[u][q], o, S);
            if (r == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (cb + u < k)
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < a.nrhs)
                                a.z[(rb + q) * a.ldz + col0 + cb + u] = acc[u][q] * sc;
            }
        }
    }
}

// one launch of level l's stage 1 with its current shape
template <int DT, int NR> void launch_s1(const S1Shape &sh, S1Args a, hipStream_t s) {
    const int grid = grid_for(a.nitems * 64, 256);
    if (sh.packed) {
#define H3D_S1P(SS, UU)                                                                   \
    if (sh.S == SS && sh.U == UU) {                                                       \
        k_s1_packed<SS, UU, DT, NR><<<grid, 256, 0, s>>>(a);                              \
        return;                                                                           \
    }
        H3D_S1P(4, 2) H3D_S1P(4, 4) H3D_S1P(8, 2) H3D_S1P(8, 4) H3D_S1P(16, 2) H3D_S1P(16, 4)
#undef H3D_S1P
    } else {
#define H3D_S1W(SS, UU)                                                                   \
    if (sh.S == SS && sh.U == UU) {                                                       \
        k_s1_wide<SS, UU, DT, NR><<<grid, 256, 0, s>>>(a);                                \
        return;                                                                           \
    }
        H3D_S1W(8, 4) H3D_S1W(8, 8) H3D_S1W(16, 4) H3D_S1W(16, 8) H3D_S1W(32, 4) H3D_S1W(32, 8)
        H3D_S1W(64, 2) H3D_S1W(64, 4) H3D_S1W(64, 8)
#undef H3D_S1W
    }
    fail(H3D_EDEVICE, "internal: no stage-1 kernel for this shape");
}

// ---------------------------------------------------------------------------
// stage 2: one workgroup per box of the chunk level, one lane per row (two
// for boxes of 65..128 rows).  At levels up to the chunk level every lane of
// the workgroup lies in the same box, so the block metadata and z are
// wave-uniform (scalar loads) and each lane streams one column slice of U per
// load, U2 loads in flight; the waves split the box's blocks.
struct S2Tab {
    int64_t box_base[kMaxLevels + 1];
    int L, lc;
};

template <int DT, int NR, int U2>
__device__ __forceinline__ void stage2_block(const typename Fac<DT>::T *__restrict__ p, int bm, int k,
                                             const double *__restrict__ zz, int64_t ldz, int rb,
                                             int nrhs, double (&acc)[NR]) {
    int c = 0;
    for (; c + U2 <= k; c += U2) {
        double v[U2];
#pragma unroll
        for (int u = 0; u < U2; ++u)
            v[u] = fac_ld<DT, kS2NonTemporal>(p + int64_t(c + u) * bm);
#pragma unroll
        for (int u = 0; u < U2; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (NR == 1 || rb + q < nrhs)
                    acc[q] += v[u] * zz[(rb + q) * ldz + c + u];
    }
    for (; c < k; ++c) {
        const double v = fac_ld<DT, kS2NonTemporal>(p + int64_t(c) * bm);
#pragma unroll
        for (int q = 0; q < NR; ++q)
            if (NR == 1 || rb + q < nrhs)
                acc[q] += v * zz[(rb + q) * ldz + c];
    }
}

// The same for two rows per lane, d rows apart (d = 0 for a lane whose second
// row lies past the box: it then repeats its first load and drops the sum).
template <int DT, int NR, int U2>
__device__ __forceinline__ void stage2_block2(const typename Fac<DT>::T *__restrict__ p, int d,
                                              int bm, int k, const double *__restrict__ zz,
                                              int64_t ldz, int rb, int nrhs, double (&a0)[NR],
                                              double (&a1)[NR]) {
    int c = 0;
    for (; c + U2 <= k; c += U2) {
        double v[U2], w[U2];
#pragma unroll
        for (int u = 0; u < U2; ++u) {
            v[u] = fac_ld<DT, kS2NonTemporal>(p + int64_t(c + u) * bm);
            w[u] = fac_ld<DT, kS2NonTemporal>(p + d + int64_t(c + u) * bm);
        }
#pragma unroll
        for (int u = 0; u < U2; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (NR == 1 || rb + q < nrhs) {
                    const double zq = zz[(rb + q) * ldz + c + u];
                    a0[q] += v[u] * zq;
                    a1[q] += w[u] * zq;
                }
    }
    for (; c < k; ++c) {
        const double v = fac_ld<DT, kS2NonTemporal>(p + int64_t(c) * bm);
        const double w = fac_ld<DT, kS2NonTemporal>(p + d + int64_t(c) * bm);
#pragma unroll
        for (int q = 0; q < NR; ++q)
            if (NR == 1 || rb + q < nrhs) {
                const double zq = zz[(rb + q) * ldz + c];
                a0[q] += v * zq;
                a1[q] += w * zq;
            }
    }
}

template <int DT, int NR, int kS2Waves>
__global__ void __launch_bounds__(512)
    k_stage2(S2Tab tab, const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ leaf_of,
             const int64_t *__restrict__ grp_begin, const int64_t *__restrict__ grp_blk,
             void *const *__restrict__ fptr, const int32_t *__restrict__ rank,
             const int64_t *__restrict__ blk_col0, const double *__restrict__ z, int64_t ldz,
             const double *yn, int64_t n, int nrhs, const int32_t *__restrict__ perm,
             void *__restrict__ yout, int64_t ldy, int io_f32, int lb, int le, double *ypart) {
    using T = typename Fac<DT>::T;
    __shared__ double part[kS2Waves][NR][64];
    const int L = tab.L, lc = tab.lc;
    // Neighbouring chunk boxes share the cache line at their common edge in
    // every coarse column they read, and workgroups are dealt to the eight
    // XCDs (each with its own L2) in turn: give each XCD a contiguous run of
    // chunk boxes so that those lines are fetched once.
    const int64_t nch = gridDim.x;
    int64_t B = blockIdx.x;
    if ((nch & 7) == 0)
        B = (B & 7) * (nch >> 3) + (B >> 3);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int shc = 3 * (L - lc);
    const int32_t r0 = leaf_off[B << shc], r1 = leaf_off[(B + 1) << shc];
    // Passes of up to 128 rows: a box of 65..128 rows reads every coarse
    // column slice in one pass, two rows per lane (rows rowb + lane and
    // rowb + 64 + lane), instead of a second pass over the same columns.
    for (int32_t rowb = r0; rowb < r1;) {
        const bool two = r1 - rowb > 64;
        const int32_t rowA = rowb + lane, rowB = rowb + 64 + lane;
        const bool actA = rowA < r1, actB = two && rowB < r1;
        const int32_t rrA = actA ? rowA : r0;
        const int dB = actB ? 64 : 0;
        for (int rb = 0; rb < nrhs; rb += NR) {
            double acc[2][NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const bool ok = wv == 0 && (NR == 1 || rb + c < nrhs);
                acc[0][c] = ok ? yn[(rb + c) * n + rrA] : 0.0;
                acc[1][c] = (ok && two) ? yn[(rb + c) * n + rrA + dB] : 0.0;
            }
            // levels whose boxes contain the whole chunk box: wave-uniform;
            // the waves of the workgroup take every kS2Waves-th block
            for (int l = lb; l <= min(lc, le); ++l) {
                const int sh = 3 * (L - l);
                const int64_t t = B >> (3 * (lc - l));
                const int64_t g = tab.box_base[l] + t;
                const int32_t bs = leaf_off[t << sh];
                const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                const int32_t loc = rrA - bs;
                const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                for (int64_t e = e0 + wv; e < e1; e += kS2Waves) {
                    const int64_t bi = grp_blk ? grp_blk[e] : e;
                    const T *p = static_cast<const T *>(fptr[bi]) + loc;
                    if (two)
                        stage2_block2<DT, NR, 8>(p, dB, bm, rank[bi], z + blk_col0[bi], ldz, rb,
                                                 nrhs, acc[0], acc[1]);
                    else
                        stage2_block<DT, NR, 8>(p, bm, rank[bi], z + blk_col0[bi], ldz, rb, nrhs,
                                                acc[0]);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && !two)
                    break;
                const int32_t row = h ? rowB : rowA;
                const bool act = h ? actB : actA;
                const int32_t rr = act ? row : r0;
                const int32_t leaf = leaf_of[rr];
                // finer levels: every lane follows the box of its own row
                for (int l = max(lc + 1, lb); l <= le; ++l) {
                    const int sh = 3 * (L - l);
                    const int64_t t = int64_t(leaf) >> sh;
                    const int64_t g = tab.box_base[l] + t;
                    const int32_t bs = leaf_off[t << sh];
                    const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                    const int32_t loc = rr - bs;
                    const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                    for (int64_t e = e0 + wv; e < e1; e += kS2Waves) {
                        const int64_t bi = grp_blk ? grp_blk[e] : e;
                        const T *p = static_cast<const T *>(fptr[bi]) + loc;
                        stage2_block<DT, NR, 4>(p, bm, rank[bi], z + blk_col0[bi], ldz, rb, nrhs,
                                                acc[h]);
                    }
                }
                // combine the waves' partial sums in a fixed order
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    part[wv][q][lane] = acc[h][q];
                __syncthreads();
                if (wv == 0) {
                    double y[NR];
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        double v = part[0][q][lane];
#pragma unroll
                        for (int w2 = 1; w2 < kS2Waves; ++w2)
                            v += part[w2][q][lane];
                        y[q] = v;
                    }
                    if (act && ypart) {
                        // partial sums in sorted order (level-by-level profiling)
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < nrhs)
                                ypart[(rb + q) * n + row] = y[q];
                    } else if (act) {
                        const int64_t dst = perm[row];
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < nrhs) {
                                if (io_f32)
                                    static_cast<float *>(yout)[(rb + q) * ldy + dst] = float(y[q]);
                                else
                                    static_cast<double *>(yout)[(rb + q) * ldy + dst] = y[q];
                            }
                    }
                }
                __syncthreads();
            }
        }
        rowb += two ? 128 : 64;
    }
}

template <int DT, int NR>
void launch_s2_kernel(int waves, int64_t nchunk, hipStream_t s, const S2Tab &tab, const Plan &P,
                      const int64_t *grp_blk, void *const *fptr, const double *z, const double *yn,
                      int nrhs, void *y, int64_t ldy, int io_f32, int lb, int le, double *ypart) {
#define H3D_S2(W)                                                                           \
    k_stage2<DT, NR, W><<<int(nchunk), 64 * W, 0, s>>>(                                     \
        tab, P.leaf_off, P.leaf_of, P.tgt_begin, grp_blk, fptr, P.blk_rank, P.blk_col0, z,  \
        P.ncols, yn, P.n, nrhs, P.perm, y, ldy, io_f32, lb, le, ypart)
    if (waves <= 2)
        H3D_S2(2);
    else if (waves <= 4)
        H3D_S2(4);
    else
        H3D_S2(8);
#undef H3D_S2
    H3D_LAUNCH_CHECK();
}

template <int DT, int NR>
S1Args stage1_args(const Plan &P, int cls, int l, bool adjoint, int nrhs, const double *xp,
                   double *z) {
    S1Args a;
    a.items = reinterpret_cast<const int2 *>(P.s1_items[cls][l]);
    a.nitems = P.s1_nitems[cls][l];
    a.span = P.s1_span[cls][l];
    a.blk_col0 = P.blk_col0;
    a.rank = P.blk_rank;
    a.seg_len = adjoint ? P.blk_m : P.blk_n;
    a.seg_off = adjoint ? P.blk_toff : P.blk_soff;
    a.seg_ptr = adjoint ? P.blk_uptr : P.blk_vptr;
    a.scale2 = P.blk_scale;
    a.nrhs = nrhs;
    a.xp = xp;
    a.n = P.n;
    a.z = z;
    a.ldz = P.ncols;
    return a;
}

template <int DT, int NR>
void launch_far(Plan &P, bool adjoint, int nrhs, const double *xp, double *z, const double *yn,
                void *y, int64_t ldy, int io_f32, hipStream_t s) {
    const int64_t n = P.n;
    const int L = P.L;
    const int cls = NR == 1 ? 0 : 1;
    const double es = DT == H3D_F64 ? 8.0 : (DT == H3D_F32 ? 4.0 : 2.0);
    // stage 1: one launch per level
    for (int l = 1; l <= L; ++l) {
        const S1Args a = stage1_args<DT, NR>(P, cls, l, adjoint, nrhs, xp, z);
        if (a.nitems == 0)
            continue;
        const S1Shape &sh = P.s1_shape[cls][l];
        const double ent = double(adjoint ? P.lvl_entries_u[l] : P.lvl_entries_v[l]);
        const double cols = double(P.lvl_rank_sum[l]);
        const double bytes = ent * es + cols * 8.0 * nrhs + double(n) * 8.0 * nrhs;
        hipEvent_t ev = P.prof.begin(s);
        launch_s1<DT, NR>(sh, a, s);
        H3D_LAUNCH_CHECK();
        char name[48];
        if (P.prof.levels)
            snprintf(name, sizeof(name), "%s_L%d", sh.packed ? "k_s1_packed" : "k_s1_wide", l);
        else
            snprintf(name, sizeof(name), "%s", sh.packed ? "k_s1_packed" : "k_s1_wide");
        P.prof.end(s, ev, name, bytes, 2.0 * ent * nrhs);
    }
    // stage 2 (always: it also writes y); level by level when profiling
    // levels, carrying the partial sums in yn
    S2Tab tab{};
    for (int l = 0; l <= kMaxLevels; ++l)
        tab.box_base[l] = P.box_base[l];
    tab.L = L;
    tab.lc = P.chunk_level;
    const int64_t nchunk = pow8(P.chunk_level);
    const int parts = (P.prof.levels && L > 1) ? L : 1;
    for (int part = 1; part <= parts; ++part) {
        const int lb = parts == 1 ? 1 : part, le = parts == 1 ? L : part;
        const bool last = part == parts;
        double ent = double(adjoint ? P.entries_v : P.stats.factor_entries - P.entries_v);
        double cols = double(P.ncols);
        if (parts > 1) {
            ent = double(adjoint ? P.lvl_entries_v[part] : P.lvl_entries_u[part]);
            cols = double(P.lvl_rank_sum[part]);
        }
        const double bytes = ent * es + cols * 8.0 * nrhs +
                             double(n) * (8.0 + (io_f32 ? 4.0 : 8.0)) * nrhs + double(n) * 8.0;
        hipEvent_t ev = P.prof.begin(s);
        launch_s2_kernel<DT, NR>(P.s2_waves[cls], nchunk, s, tab, P, adjoint ? P.src_blk : nullptr,
                                 adjoint ? P.blk_vptr : P.blk_uptr, z, yn, nrhs, y, ldy, io_f32,
                                 lb, le, last ? nullptr : const_cast<double *>(yn));
        char name[48];
        if (parts > 1)
            snprintf(name, sizeof(name), "k_stage2_L%d", part);
        else
            snprintf(name, sizeof(name), "k_stage2");
        P.prof.end(s, ev, name, bytes, 2.0 * ent * nrhs);
    }
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate stage-1 shapes level by level and stage-2 wave
// counts on the plan's own factor streams, keeps the fastest of each.
std::vector<S1Shape> s1_candidates(const Plan &P, int l) {
    std::vector<S1Shape> c;
    const int m = std::max(1, P.mean_box[l]);
    auto add = [&](int packed, int S, int U, int reps) {
        S1Shape sh;
        sh.packed = packed;
        sh.S = S;
        sh.U = U;
        sh.reps = reps;
        c.push_back(sh);
    };
    if (m <= 32) {
        add(1, 4, 2, 1);
        add(1, 4, 4, 1);
        add(1, 8, 2, 1);
        add(1, 8, 4, 1);
    }
    if (m >= 8 && m <= 128) {
        add(1, 16, 2, 1);
        add(1, 16, 4, 1);
    }
    for (int S : {8, 16, 32, 64}) {
        if (S > std::max(8, 2 * m) || 16 * S < m)
            continue;
        for (int U : {4, 8}) {
            add(0, S, U, 1);
            add(0, S, U, 64);
        }
        if (S == 64)
            add(0, 64, 2, 1);
    }
    return c;
}

template <int DT, int NR>
void autotune_dt(Plan &P, int nrhs, hipStream_t s) {
    const int cls = NR == 1 ? 0 : 1;
    hipEvent_t e0, e1;
    H3D_HIP(hipEventCreate(&e0));
    H3D_HIP(hipEventCreate(&e1));
    auto time_it = [&](auto &&launch) {
        launch();  // warm-up
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            H3D_HIP(hipEventRecord(e0, s));
            launch();
            H3D_HIP(hipEventRecord(e1, s));
            H3D_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            H3D_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return best;
    };
    for (int l = 1; l <= P.L; ++l) {
        if (P.lvl_blk[l + 1] <= P.lvl_blk[l])
            continue;
        S1Shape best_sh = P.s1_shape[cls][l];
        float best_ms = 1e30f;
        for (const S1Shape &sh : s1_candidates(P, l)) {
            set_level_shape(P, cls, l, sh, s);
            const S1Args a = stage1_args<DT, NR>(P, cls, l, false, nrhs, P.xp, P.z);
            const float ms = time_it([&] { launch_s1<DT, NR>(sh, a, s); });
            if (ms < best_ms) {
                best_ms = ms;
                best_sh = sh;
            }
        }
        set_level_shape(P, cls, l, best_sh, s);
    }
    S2Tab tab{};
    for (int l = 0; l <= kMaxLevels; ++l)
        tab.box_base[l] = P.box_base[l];
    tab.L = P.L;
    tab.lc = P.chunk_level;
    const int64_t nchunk = pow8(P.chunk_level);
    float best_ms = 1e30f;
    int best_w = P.s2_waves[cls];
    for (int w : {2, 4, 8}) {
        const float ms = time_it([&] {
            launch_s2_kernel<DT, NR>(w, nchunk, s, tab, P, nullptr, P.blk_uptr, P.z, P.yp, nrhs,
                                     P.yp + P.n * nrhs, P.n, 0, 1, P.L, nullptr);
        });
        if (ms < best_ms) {
            best_ms = ms;
            best_w = w;
        }
    }
    P.s2_waves[cls] = best_w;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P.tuned[cls] = true;
}

template <int NR>
void launch_near(Plan &P, int nrhs, const double *xp, double *yn, hipStream_t s) {
    hipEvent_t ev = P.prof.begin(s);
    k_near<NR><<<int(pow8(P.L)), 64, 0, s>>>(P.L, P.leaf_off, P.near_ptr, P.near_s, P.px, P.py,
                                              P.pz, P.cfg.kernel, P.cfg.kernel_param, nrhs, xp,
                                              P.n, yn);
    H3D_LAUNCH_CHECK();
    P.prof.end(s, ev, "k_near", double(P.n) * (32.0 + 8.0 * nrhs),
               double(P.stats.near_pair_evals) * (10.0 + 2.0 * nrhs));
}

}  // namespace

static void ensure_scratch(Plan &P, int64_t nrhs, hipStream_t s) {
    if (nrhs <= P.scratch_nrhs)
        return;
    const int64_t n = P.n;
    P.mem.release(P.xp);
    P.mem.release(P.yp);
    P.mem.release(P.z);
    P.xp = P.mem.alloc_n<double>(n * nrhs);
    P.yp = P.mem.alloc_n<double>(2 * n * nrhs);  // second half: tuner output
    P.z = P.mem.alloc_n<double>(std::max<int64_t>(P.ncols, 1) * nrhs);
    H3D_HIP(hipMemsetAsync(P.xp, 0, sizeof(double) * size_t(n * nrhs), s));
    H3D_HIP(hipMemsetAsync(P.yp, 0, sizeof(double) * size_t(2 * n * nrhs), s));
    P.scratch_nrhs = nrhs;
}

void autotune(Plan &P, int64_t nrhs, hipStream_t s) {
    if (P.nfar == 0 || nrhs >= kBatchedMinRhs)
        return;
    const int nr = nrhs == 1 ? 1 : int(std::min<int64_t>(nrhs, 4));
    ensure_scratch(P, std::max<int64_t>(nrhs, nr), s);
    auto go = [&](auto dt_tag) {
        constexpr int DT = decltype(dt_tag)::value;
        if (nrhs == 1)
            autotune_dt<DT, 1>(P, 1, s);
        else
            autotune_dt<DT, 4>(P, int(nrhs), s);
    };
    switch (P.factor_dtype) {
    case H3D_F64:
        go(std::integral_constant<int, H3D_F64>{});
        break;
    case H3D_F32:
        go(std::integral_constant<int, H3D_F32>{});
        break;
    default:
        go(std::integral_constant<int, H3D_BF16_SCALED>{});
        break;
    }
    H3D_HIP(hipStreamSynchronize(s));
}

void matvec_run(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                int io_dtype, bool adjoint, hipStream_t s) {
    if (nrhs >= kBatchedMinRhs) {
        matvec_batched(P, x, y, nrhs, ldx, ldy, io_dtype, adjoint, s);
        return;
    }
    const int64_t n = P.n;
    ensure_scratch(P, nrhs, s);
    const int io_f32 = io_dtype == H3D_F32;
    {
        hipEvent_t ev = P.prof.begin(s);
        k_gather<<<grid_for(n, 256), 256, 0, s>>>(x, io_f32, ldx, n, int(nrhs), P.perm, P.xp);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "k_gather", double(n) * (4.0 + (io_f32 ? 4.0 : 8.0) * nrhs + 8.0 * nrhs), 0.0);
    }
    // The near list is symmetric (t in Near(s) iff s in Near(t)), and the
    // kernels are radial, so K(t,s)^T = K(s,t): the adjoint near field walks
    // the same list with the roles of row and column exchanged.
    if (nrhs == 1)
        launch_near<1>(P, 1, P.xp, P.yp, s);
    else
        launch_near<4>(P, int(nrhs), P.xp, P.yp, s);
    auto far = [&](auto dt_tag) {
        constexpr int DT = decltype(dt_tag)::value;
        if (nrhs == 1)
            launch_far<DT, 1>(P, adjoint, 1, P.xp, P.z, P.yp, y, ldy, io_f32, s);
        else
            launch_far<DT, 4>(P, adjoint, int(nrhs), P.xp, P.z, P.yp, y, ldy, io_f32, s);
    };
    switch (P.factor_dtype) {
    case H3D_F64:
        far(std::integral_constant<int, H3D_F64>{});
        break;
    case H3D_F32:
        far(std::integral_constant<int, H3D_F32>{});
        break;
    default:
        far(std::integral_constant<int, H3D_BF16_SCALED>{});
        break;
    }
}

}  // namespace h3d
