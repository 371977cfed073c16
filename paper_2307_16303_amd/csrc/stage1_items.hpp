// Stage-1 work items of the mat-vec (Algorithm 2, low-rank part): the dot
// products z = V_b^T x_s (in the adjoint U_b^T x_t) of one item of a level.
// Called by the per-level stage-1 kernels of a single operator and by the
// stage-1 launches of a batch of operators.
#pragma once

#include "product_items.hpp"

namespace h3d {
namespace dev {

// v + the value of the lane given by a DPP row permutation (CTRL), on both
// halves of a double
template <int CTRL> __device__ __forceinline__ double dpp_add(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return v + __hiloint2double(hi, lo);
}

// Sum over aligned groups of S <= 16 lanes, the same value in every lane of
// the group: swap neighbours, swap pairs (quad permutations), then mirror the
// half row and the row, each step adding a partial sum of the other half.
template <int S> __device__ __forceinline__ double group_sum(double v) {
    if constexpr (S >= 2)
        v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
    if constexpr (S >= 4)
        v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (S >= 8)
        v = dpp_add<0x141>(v);  // row_half_mirror
    if constexpr (S >= 16)
        v = dpp_add<0x140>(v);  // row_mirror
    static_assert(S <= 16, "DPP row permutations cover 16 lanes");
    return v;
}

// Sum over aligned sub-waves of S lanes, the same value in every lane: DPP
// row permutations within rows of 16 lanes, shuffles for the wider strides.
template <int S> __device__ __forceinline__ double sub_sum(double v) {
    v = group_sum<(S < 16 ? S : 16)>(v);
#pragma unroll
    for (int o = 16; o < S; o <<= 1)
        v += __shfl_xor(v, o, S);
    return v;
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
    // split columns (wide form, one RHS): part of each item, rows per part,
    // and the partial sums (span per item)
    const int32_t *part;
    int rows;
    double *zp;
};

// item w of a level: (block, first column), one 8-byte global load
__device__ __forceinline__ int2 item_of(const int2 *items, int64_t w) {
    const uint64_t v = glob(reinterpret_cast<const uint64_t *>(items))[w];
    return make_int2(int(uint32_t(v)), int(uint32_t(v >> 32)));
}

template <int S, int U, int DT, int NR>
__device__ __forceinline__ void s1_wide_item(const S1Args &a, int64_t w) {
    using T = typename Fac<DT>::T;
    constexpr int NS = 64 / S;
    const int2 item = item_of(a.items, w);
    const int lane = threadIdx.x & 63;
    const int r = lane % S, sub = lane / S;
    const int b = item.x;
    const int len = glob(a.seg_len)[b];
    const int64_t off = glob(a.seg_off)[b];
    const int64_t col0 = glob(a.blk_col0)[b];
    const int k = glob(a.rank)[b];
    const T *__restrict__ p = static_cast<const T *>(glob(a.seg_ptr)[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(glob(a.scale2)[2 * b]) * double(glob(a.scale2)[2 * b + 1]);
    const int cend = min(item.y + a.span, k);
    const auto xp = glob(a.xp);
    // rows of this item: a part of the column when columns are split
    int j0 = 0, j1 = len;
    if (a.part) {
        j0 = glob(a.part)[w] * a.rows;
        j1 = min(len, j0 + a.rows);
    }
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        for (int cb = item.y; cb < cend; cb += NS * U) {
            double acc[U][NR];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] = 0.0;
            // JU rows per round (one right-hand side, FP32/BF16 factors, whose
            // loads are narrow), so that one round keeps about 16 loads in
            // flight (measured slower for FP64): every load is issued, from a row of the
            // item and a column clamped into the item (cend > cb here); rows
            // past the item's end take x = 0, columns past it drop the value
            constexpr int JU = NR == 1 && DT != H3D_F64 && U < 16 ? 16 / U : 1;
            for (int jb = j0 + r; jb < j1; jb += S * JU) {
                double xv[JU][NR];
                T vr[JU][U];
#pragma unroll
                for (int i = 0; i < JU; ++i) {
                    const int j = jb + i * S, jc = min(j, j1 - 1);
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const double xr = (NR == 1 || rb + q < a.nrhs)
                                              ? xp[(rb + q) * a.n + off + jc]
                                              : 0.0;
                        xv[i][q] = j < j1 ? xr : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        vr[i][u] =
                            fac_raw<DT>(p + int64_t(min(cb + sub + u * NS, cend - 1)) * len + jc);
                }
#pragma unroll
                for (int i = 0; i < JU; ++i)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const double v = cb + sub + u * NS < cend ? Fac<DT>::cvt(vr[i][u]) : 0.0;
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            acc[u][q] += v * xv[i][q];
                    }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] = sub_sum<S>(acc[u][q]);
            if (r == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = cb + sub + u * NS;
                    if (a.part)  // one pass of span columns per item
                        glob(a.zp)[w * int64_t(a.span) + (c - item.y)] = acc[u][0] * sc;
                    else if (c < cend)
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < a.nrhs)
                                glob(a.z)[(rb + q) * a.ldz + col0 + c] = acc[u][q] * sc;
                }
            }
        }
    }
}

template <int S, int U, int DT, int NR>
__device__ __forceinline__ void s1_packed_item(const S1Args &a, int64_t w) {
    using T = typename Fac<DT>::T;
    const int2 item = item_of(a.items, w);
    const int lane = threadIdx.x & 63;
    const int r = lane % S, sub = lane / S;
    const bool valid = sub < item.y;
    const int b = item.x + (valid ? sub : 0);
    const int k = valid ? glob(a.rank)[b] : 0;
    const int len = k > 0 ? glob(a.seg_len)[b] : 0;  // no rows, so no loads, without columns
    const int64_t off = glob(a.seg_off)[b];
    const int64_t col0 = glob(a.blk_col0)[b];
    const T *__restrict__ p = static_cast<const T *>(glob(a.seg_ptr)[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(glob(a.scale2)[2 * b]) * double(glob(a.scale2)[2 * b + 1]);
    int kmax = k;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const auto xp = glob(a.xp);
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        for (int cb = 0; cb < kmax; cb += U) {
            double acc[U][NR];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] = 0.0;
            const int jend = cb < k ? len : 0;  // this block's columns are done
            // JU rows per round as in the wide form; k > cb here, so columns
            // are clamped into the block and every load is issued
            constexpr int JU = NR == 1 && DT != H3D_F64 && U < 16 ? 16 / U : 1;
            for (int jb = r; jb < jend; jb += S * JU) {
                double xv[JU][NR];
                T vr[JU][U];
#pragma unroll
                for (int i = 0; i < JU; ++i) {
                    const int j = jb + i * S, jc = min(j, jend - 1);
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const double xr = (NR == 1 || rb + q < a.nrhs)
                                              ? xp[(rb + q) * a.n + off + jc]
                                              : 0.0;
                        xv[i][q] = j < jend ? xr : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        vr[i][u] = fac_raw<DT>(p + int64_t(min(cb + u, k - 1)) * len + jc);
                }
#pragma unroll
                for (int i = 0; i < JU; ++i)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const double v = cb + u < k ? Fac<DT>::cvt(vr[i][u]) : 0.0;
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            acc[u][q] += v * xv[i][q];
                    }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] = sub_sum<S>(acc[u][q]);
            if (r == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (cb + u < k)
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < a.nrhs)
                                glob(a.z)[(rb + q) * a.ldz + col0 + cb + u] = acc[u][q] * sc;
            }
        }
    }
}

// Adjoint stage 1 above the chunk level: z_c = (column c of U_b) . x_t with
// U_b stored as row panels.  Item = (block, first column); a wave takes
// kPanelCols columns side by side over 64 lanes per column and walks the
// panels of the target box in row order.
constexpr int kPanelCols = 8;

template <int DT, int NR>
__device__ __forceinline__ void s1_panel_item(const S1Args &a, const int32_t *__restrict__ leaf_off,
                                              const int32_t *__restrict__ box, int shc, int shl,
                                              int64_t w) {
    using T = typename Fac<DT>::T;
    constexpr int U = kPanelCols;
    const int2 item = a.items[w];
    const int lane = threadIdx.x & 63;
    const int b = item.x;
    const int32_t bs = a.seg_off[b];
    const int64_t col0 = a.blk_col0[b];
    const int k = a.rank[b];
    const T *__restrict__ p = static_cast<const T *>(a.seg_ptr[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(a.scale2[2 * b]) * double(a.scale2[2 * b + 1]);
    const int cb = item.y;
    const int64_t ch0 = int64_t(box[b]) << shl, nch = int64_t(1) << shl;
    const double *__restrict__ xp = a.xp;
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        double acc[U][NR];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                acc[u][q] = 0.0;
        for (int64_t ch = ch0; ch < ch0 + nch; ++ch) {
            const int32_t r0 = leaf_off[ch << shc], r1 = leaf_off[(ch + 1) << shc];
            const int mj = r1 - r0;
            const T *__restrict__ pj = p + int64_t(r0 - bs) * k;
            for (int j = lane; j < mj; j += 64) {
                double xv[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    xv[q] = (NR == 1 || rb + q < a.nrhs) ? xp[(rb + q) * a.n + r0 + j]
                                                         : 0.0;
                // cb < k: columns clamped into the block, every load issued
                T vr[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    vr[u] = fac_raw<DT>(pj + int64_t(min(cb + u, k - 1)) * mj + j);
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    v[u] = cb + u < k ? Fac<DT>::cvt(vr[u]) : 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        acc[u][q] += v[u] * xv[q];
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    acc[u][q] += __shfl_xor(acc[u][q], o, 64);
        if (lane == 0) {
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

// Split columns: column u of column group g of a level gets the sum of its
// parts' partial sums, added in part order (grp[2 g] = the group's first item,
// grp[2 g + 1] = its part count; one thread per (group, column)).
__device__ __forceinline__ void s1_reduce_column(int64_t t, int64_t ngrp,
                                                 const int32_t *__restrict__ grp,
                                                 const S1Args &a) {
    const int64_t g = t / a.span;
    const int u = int(t - g * a.span);
    if (g >= ngrp)
        return;
    const int32_t first = glob(grp)[2 * g], np = glob(grp)[2 * g + 1];
    const int2 it = item_of(a.items, first);
    if (it.y + u >= glob(a.rank)[it.x])
        return;
    double v = 0.0;
    for (int32_t pp = 0; pp < np; ++pp)
        v += glob(a.zp)[int64_t(first + pp) * a.span + u];
    glob(a.z)[glob(a.blk_col0)[it.x] + it.y + u] = v;
}

}  // namespace dev
}  // namespace h3d
