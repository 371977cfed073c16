// Finest level of a one-right-hand-side product with both stages of
// Algorithm 2 fused (k_leaf); the product driver decides when it runs.
#include "stage1_items.hpp"

namespace h3d {

namespace {

using namespace dev;

// Finest level, one right-hand side: both stages of Algorithm 2 for the far
// blocks of one output leaf o, one wave per leaf,
//     y_o += sum_b A_b (B_b^T x_i(b)),
// with A_b = U_b, B_b = V_b and i(b) the source leaf in a forward product
// (blocks grouped by target), and A_b = V_b, B_b = U_b, i(b) the target leaf in
// the adjoint (blocks grouped by source through grp_blk).  The wave is cut into
// 64/S groups of S lanes; group g takes the blocks g, g + 64/S, ... of the
// leaf's list and, column by column, forms z_c = B_b[:, c] . x_i (S lanes over
// the rows of the input leaf, reduced within the group) and adds A_b[:, c] z_c
// to its partial sums of the rows of y_o, so z never leaves the registers.
// Which block a group takes depends only on its position in the list, so the
// sums do not depend on where the factors are stored.  A group keeps UR
// columns in flight; rows of y_o are taken kLeafRows at a time (a taller leaf
// repeats the pass).

struct LeafArgs {
    int64_t nleaf;
    const int64_t *grp_begin;  // [nleaf + 1] block range of each output leaf
    const int64_t *grp_blk;    // block ids in group order, or NULL (identity)
    const int32_t *leaf_off;
    void *const *aptr;         // A_b: rows of the output leaf x k, column-major
    void *const *bptr;         // B_b: rows of the input leaf x k, column-major
    const int32_t *rank;
    const int32_t *in_len, *in_off;  // rows of the input leaf of each block
    const float *scale2;
    const double *xp;          // sorted input
    double *yn;                // sorted partial sums, updated in place
};

// Global-memory load of a factor entry through a pointer that the compiler
// cannot place itself (it was read from LDS): without the address space the
// load would be a flat one, which also waits on the LDS counter.
template <int DT, int S, int UR>
__global__ void __launch_bounds__(256) k_leaf(LeafArgs a) {
    using T = typename Fac<DT>::T;
    constexpr int G = 64 / S, RM = kLeafRows / S;
    __shared__ int32_t s_k[4][64], s_len[4][64], s_off[4][64];
    __shared__ const T *s_a[4][64];
    __shared__ const T *s_b[4][64];
    __shared__ float s_sc[4][64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t o = int64_t(blockIdx.x) * 4 + wv;
    if (o >= a.nleaf)
        return;  // the whole wave; nothing below synchronises the workgroup
    const int g = lane / S, r = lane % S;
    const int32_t r0 = a.leaf_off[o], mo = a.leaf_off[o + 1] - r0;
    const int64_t e0 = a.grp_begin[o], e1 = a.grp_begin[o + 1];
    for (int ro = 0; ro < mo; ro += kLeafRows) {
        double acc[RM];
#pragma unroll
        for (int h = 0; h < RM; ++h)
            acc[h] = 0.0;
        for (int64_t q = e0; q < e1; q += 64) {
            // ranks, input rows and factor pointers of the next 64 blocks
            const int64_t e = q + lane;
            if (e < e1) {
                const int64_t bi = a.grp_blk ? a.grp_blk[e] : e;
                s_k[wv][lane] = a.rank[bi];
                s_len[wv][lane] = a.in_len[bi];
                s_off[wv][lane] = a.in_off[bi];
                s_a[wv][lane] = static_cast<const T *>(a.aptr[bi]);
                s_b[wv][lane] = static_cast<const T *>(a.bptr[bi]);
                if (DT == H3D_BF16_SCALED)
                    s_sc[wv][lane] = a.scale2[2 * bi] * a.scale2[2 * bi + 1];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int nb = int(min<int64_t>(64, e1 - q));
            for (int jb = g; jb < nb; jb += G) {
                const int k = s_k[wv][jb], len = s_len[wv][jb];
                const T *ap = s_a[wv][jb], *bp = s_b[wv][jb];
                const double *xq = a.xp + s_off[wv][jb];
                // Every block has m, n >= 1, and k >= 1 inside the column loop:
                // indexes are clamped into the block, so every load is issued
                // unconditionally, and lanes off the block then drop the value.
                // A lane takes the input rows r + h S (h < RM) of each column,
                // and any further rows of a taller leaf in a loop.
                int rv[RM];
                double x0[RM];
#pragma unroll
                for (int h = 0; h < RM; ++h) {
                    rv[h] = min(r + h * S, len - 1);
                    x0[h] = r + h * S < len ? xq[rv[h]] : 0.0;
                }
                for (int c = 0; c < k; c += UR) {
                    T vr[UR][RM], ur[UR][RM];
#pragma unroll
                    for (int t = 0; t < UR; ++t) {
                        const int64_t cc = min(c + t, k - 1);
#pragma unroll
                        for (int h = 0; h < RM; ++h)
                            vr[t][h] = fac_raw<DT>(bp + cc * len + rv[h]);
#pragma unroll
                        for (int h = 0; h < RM; ++h)
                            if (ro + h * S < mo)  // wave-uniform
                                ur[t][h] = fac_raw<DT>(ap + cc * mo + min(ro + h * S + r, mo - 1));
                    }
#pragma unroll
                    for (int t = 0; t < UR; ++t) {
                        const bool on = c + t < k;
                        double zs = 0.0;
#pragma unroll
                        for (int h = 0; h < RM; ++h)
                            zs += on ? Fac<DT>::cvt(vr[t][h]) * x0[h] : 0.0;
                        if (len > kLeafRows && on)
                            for (int jr = r + kLeafRows; jr < len; jr += S)
                                zs += fac_ld<DT>(bp + int64_t(c + t) * len + jr) * xq[jr];
                        zs = group_sum<S>(zs);
                        if (DT == H3D_BF16_SCALED)
                            zs *= double(s_sc[wv][jb]);
#pragma unroll
                        for (int h = 0; h < RM; ++h)
                            if (ro + h * S < mo) {
                                const bool rin = on && ro + h * S + r < mo;
                                acc[h] += (rin ? Fac<DT>::cvt(ur[t][h]) : 0.0) * zs;
                            }
                    }
                }
            }
            // every lane has read this chunk's entries before the next overwrites them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int h = 0; h < RM; ++h)
#pragma unroll
            for (int d = S; d < 64; d <<= 1)
                acc[h] += __shfl_xor(acc[h], d, 64);
        if (g == 0)
#pragma unroll
            for (int h = 0; h < RM; ++h) {
                const int row = ro + h * S + r;
                if (row < mo)
                    a.yn[r0 + row] += acc[h];
            }
    }
}

template <int DT>
void launch_leaf_dt(const Plan &P, int shape, bool adjoint, const double *xp, double *yn,
                    hipStream_t s) {
    LeafArgs a{};
    a.nleaf = pow8(P.L);
    a.grp_begin = P.tgt_begin + P.box_base[P.L];
    a.grp_blk = adjoint ? P.src_blk : nullptr;
    a.leaf_off = P.leaf_off;
    a.aptr = adjoint ? P.blk_vptr : P.blk_uptr;
    a.bptr = adjoint ? P.blk_uptr : P.blk_vptr;
    a.rank = P.blk_rank;
    a.in_len = adjoint ? P.blk_m : P.blk_n;
    a.in_off = adjoint ? P.blk_toff : P.blk_soff;
    a.scale2 = P.blk_scale;
    a.xp = xp;
    a.yn = yn;
    const int grid = int((a.nleaf + 3) / 4);
    switch (shape) {
#define H3D_LEAF(S_, U_)                                                                    \
    case (S_) | ((U_) << 8):                                                                \
        k_leaf<DT, S_, U_><<<grid, 256, 0, s>>>(a);                                         \
        break;
        H3D_LEAF(8, 2)
        H3D_LEAF(8, 3)
        H3D_LEAF(16, 2)
        H3D_LEAF(16, 3)
#undef H3D_LEAF
    default:
        fail(H3D_EINVAL, "internal: unknown leaf launch shape");
    }
    H3D_LAUNCH_CHECK();
}


}  // namespace

int leaf_shape(const Plan &P) {
    if (P.in_batch || P.L < 1 || P.lvl_blk[P.L + 1] <= P.lvl_blk[P.L])
        return 0;
    if (P.leaf_fuse >= 0)
        return P.leaf_fuse;
    return P.mean_box[P.L] <= kLeafRows ? (8 | (3 << 8)) : 0;
}

std::vector<int> leaf_candidates() {
    return {0, 8 | (2 << 8), 8 | (3 << 8), 16 | (2 << 8), 16 | (3 << 8)};
}

void launch_leaf(const Plan &P, int shape, bool adjoint, const double *xp, double *yn,
                 hipStream_t s) {
    switch (P.factor_dtype) {
    case H3D_F64:
        launch_leaf_dt<H3D_F64>(P, shape, adjoint, xp, yn, s);
        break;
    case H3D_F32:
        launch_leaf_dt<H3D_F32>(P, shape, adjoint, xp, yn, s);
        break;
    default:
        launch_leaf_dt<H3D_BF16_SCALED>(P, shape, adjoint, xp, yn, s);
        break;
    }
}

}  // namespace h3d
