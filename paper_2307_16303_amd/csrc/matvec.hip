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
// Stage 2 gives every row its own lane: one wave per box of a chunk level
// (boxes of roughly 64 points), looping over the levels; at each level the
// lane streams the column slices of the factors of the box that contains its
// row.  No atomics: every output row is written by exactly one lane, and the
// summation order is fixed, so results are bitwise reproducible.
#include "h3d_internal.hpp"

namespace h3d {

namespace {

template <int DT> struct Fac;
template <> struct Fac<H3D_F64> {
    using T = double;
    static __device__ __forceinline__ double ld(const T *p) { return __builtin_nontemporal_load(p); }
};
template <> struct Fac<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ double ld(const T *p) { return double(__builtin_nontemporal_load(p)); }
};
template <> struct Fac<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ double ld(const T *p) {
        return double(__uint_as_float(uint32_t(__builtin_nontemporal_load(p)) << 16));
    }
};

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
// stage 1: z[col] = dot(column col of its block's factor, x segment)
struct S1Level {
    int64_t c0, c1;  // columns of this level
    int64_t w0;      // first wave of this level
    int S;           // lanes per column
};
struct S1Tab {
    S1Level lv[kMaxLevels + 1];
    int nlev;
};

template <int S, int DT, int NR>
__device__ __forceinline__ void stage1_cols(int64_t wave, const S1Level &L, const int32_t *__restrict__ col_blk,
                                            const int64_t *__restrict__ blk_col0,
                                            const int32_t *__restrict__ seg_len,
                                            const int32_t *__restrict__ seg_off,
                                            void *const *__restrict__ seg_ptr,
                                            const float *__restrict__ scale2, int nrhs,
                                            const double *__restrict__ xp, int64_t n,
                                            double *__restrict__ z, int64_t ldz) {
    using T = typename Fac<DT>::T;
    const int lane = threadIdx.x & 63;
    const int r = lane % S;
    const int64_t col = L.c0 + wave * (64 / S) + lane / S;
    const bool act = col < L.c1;
    int len = 0;
    int64_t off = 0;
    const T *p = nullptr;
    double sc = 1.0;
    if (act) {
        const int32_t b = col_blk[col];
        len = seg_len[b];
        off = seg_off[b];
        p = static_cast<const T *>(seg_ptr[b]) + (col - blk_col0[b]) * len;
        if (DT == H3D_BF16_SCALED)
            sc = double(scale2[2 * b]) * double(scale2[2 * b + 1]);
    }
    for (int rb = 0; rb < nrhs; rb += NR) {
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            acc[c] = 0.0;
        if (act) {
            for (int j = r; j < len; j += S) {
                const double v = Fac<DT>::ld(p + j);
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (NR == 1 || rb + c < nrhs)
                        acc[c] += v * xp[(rb + c) * n + off + j];
            }
        }
#pragma unroll
        for (int o = S / 2; o > 0; o >>= 1)
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] += __shfl_xor(acc[c], o, S);
        if (act && r == 0)
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (NR == 1 || rb + c < nrhs)
                    z[(rb + c) * ldz + col] = acc[c] * sc;
    }
}

template <int DT, int NR>
__global__ void __launch_bounds__(256)
    k_stage1(S1Tab tab, int64_t nwaves, const int32_t *__restrict__ col_blk,
             const int64_t *__restrict__ blk_col0, const int32_t *__restrict__ seg_len,
             const int32_t *__restrict__ seg_off, void *const *__restrict__ seg_ptr,
             const float *__restrict__ scale2, int nrhs, const double *__restrict__ xp, int64_t n,
             double *__restrict__ z, int64_t ldz) {
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (wave >= nwaves)
        return;
    int li = 0;
    while (li + 1 < tab.nlev && wave >= tab.lv[li + 1].w0)
        ++li;
    const S1Level L = tab.lv[li];
    const int64_t w = wave - L.w0;
    switch (L.S) {
    case 4:
        stage1_cols<4, DT, NR>(w, L, col_blk, blk_col0, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    case 8:
        stage1_cols<8, DT, NR>(w, L, col_blk, blk_col0, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    case 16:
        stage1_cols<16, DT, NR>(w, L, col_blk, blk_col0, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    case 32:
        stage1_cols<32, DT, NR>(w, L, col_blk, blk_col0, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    default:
        stage1_cols<64, DT, NR>(w, L, col_blk, blk_col0, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    }
}

// ---------------------------------------------------------------------------
// stage 2: one wave per box of the chunk level, one lane per row
struct S2Tab {
    int64_t box_base[kMaxLevels + 1];
    int L, lc;
};

template <int DT, int NR>
__global__ void __launch_bounds__(256)
    k_stage2(S2Tab tab, const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ leaf_of,
             const int64_t *__restrict__ grp_begin, const int64_t *__restrict__ grp_blk,
             void *const *__restrict__ fptr, const int32_t *__restrict__ rank,
             const int64_t *__restrict__ blk_col0, const double *__restrict__ z, int64_t ldz,
             const double *__restrict__ yn, int64_t n, int nrhs, const int32_t *__restrict__ perm,
             void *__restrict__ yout, int64_t ldy, int io_f32) {
    using T = typename Fac<DT>::T;
    const int L = tab.L, lc = tab.lc;
    const int64_t B = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (B >= (int64_t(1) << (3 * lc)))
        return;
    const int shc = 3 * (L - lc);
    const int32_t r0 = leaf_off[B << shc], r1 = leaf_off[(B + 1) << shc];
    for (int32_t rowb = r0; rowb < r1; rowb += 64) {
        const int32_t row = rowb + lane;
        const bool act = row < r1;
        const int32_t rr = act ? row : r0;
        const int32_t leaf = leaf_of[rr];
        for (int rb = 0; rb < nrhs; rb += NR) {
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = (NR == 1 || rb + c < nrhs) ? yn[(rb + c) * n + rr] : 0.0;
            for (int l = 1; l <= L; ++l) {
                const int sh = 3 * (L - l);
                const int64_t t = int64_t(leaf) >> sh;
                const int64_t g = tab.box_base[l] + t;
                const int32_t bs = leaf_off[t << sh];
                const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                const int32_t loc = rr - bs;
                const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                for (int64_t e = e0; e < e1; ++e) {
                    const int64_t bi = grp_blk ? grp_blk[e] : e;
                    const int k = rank[bi];
                    const int64_t c0 = blk_col0[bi];
                    const T *p = static_cast<const T *>(fptr[bi]) + loc;
                    for (int c = 0; c < k; ++c) {
                        const double v = Fac<DT>::ld(p + int64_t(c) * bm);
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < nrhs)
                                acc[q] += v * z[(rb + q) * ldz + c0 + c];
                    }
                }
            }
            if (act) {
                const int64_t dst = perm[row];
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    if (NR == 1 || rb + q < nrhs) {
                        if (io_f32)
                            static_cast<float *>(yout)[(rb + q) * ldy + dst] = float(acc[q]);
                        else
                            static_cast<double *>(yout)[(rb + q) * ldy + dst] = acc[q];
                    }
            }
        }
    }
}

int pick_subwave(int mean) {
    int S = 4;
    while (S < 64 && S < mean)
        S *= 2;
    return S;
}

template <int DT, int NR>
void launch_far(Plan &P, bool adjoint, int nrhs, const double *xp, double *z, const double *yn,
                void *y, int64_t ldy, int io_f32, hipStream_t s) {
    const int64_t n = P.n;
    const int L = P.L;
    const size_t es = DT == H3D_F64 ? 8 : (DT == H3D_F32 ? 4 : 2);
    // stage 1
    if (P.ncols > 0) {
        S1Tab tab{};
        int64_t w = 0;
        int nl = 0;
        for (int l = 1; l <= L; ++l) {
            S1Level lv;
            lv.c0 = P.lvl_col[l];
            lv.c1 = P.lvl_col[l + 1];
            lv.S = pick_subwave(P.mean_box[l]);
            lv.w0 = w;
            w += ceil_div(lv.c1 - lv.c0, 64 / lv.S);
            tab.lv[nl++] = lv;
        }
        tab.nlev = nl;
        hipEvent_t ev = P.prof.begin(s);
        const int32_t *len = adjoint ? P.blk_m : P.blk_n;
        const int32_t *off = adjoint ? P.blk_toff : P.blk_soff;
        void *const *ptr = adjoint ? P.blk_uptr : P.blk_vptr;
        k_stage1<DT, NR><<<grid_for(w * 64, 256), 256, 0, s>>>(tab, w, P.col_blk, P.blk_col0, len,
                                                                off, ptr, P.blk_scale, nrhs, xp, n,
                                                                z, P.ncols);
        H3D_LAUNCH_CHECK();
        const double side_entries =
            double(adjoint ? P.stats.factor_entries - P.entries_v : P.entries_v);
        const double bytes = side_entries * double(es) + double(P.ncols) * 8.0 * nrhs +
                             double(n) * 8.0 * nrhs * L;
        P.prof.end(s, ev, adjoint ? "far_stage1_adj" : "far_stage1", bytes,
                   2.0 * side_entries * nrhs);
    }
    // stage 2 (always: it also writes y)
    {
        int lc = L;
        while (lc > 0 && P.mean_box[lc] < 48)
            --lc;
        S2Tab tab{};
        for (int l = 0; l <= kMaxLevels; ++l)
            tab.box_base[l] = P.box_base[l];
        tab.L = L;
        tab.lc = lc;
        hipEvent_t ev = P.prof.begin(s);
        const int64_t nchunk = pow8(lc);
        k_stage2<DT, NR><<<grid_for(nchunk * 64, 256), 256, 0, s>>>(
            tab, P.leaf_off, P.leaf_of, P.tgt_begin, adjoint ? P.src_blk : nullptr,
            adjoint ? P.blk_vptr : P.blk_uptr, P.blk_rank, P.blk_col0, z, P.ncols, yn, n, nrhs,
            P.perm, y, ldy, io_f32);
        H3D_LAUNCH_CHECK();
        const double side_entries =
            double(adjoint ? P.entries_v : P.stats.factor_entries - P.entries_v);
        const double bytes = side_entries * double(es) + double(P.ncols) * 8.0 * nrhs +
                             double(n) * (8.0 + (io_f32 ? 4.0 : 8.0)) * nrhs + double(n) * 8.0;
        P.prof.end(s, ev, adjoint ? "far_stage2_adj" : "far_stage2", bytes,
                   2.0 * side_entries * nrhs);
    }
}

template <int NR>
void launch_near(Plan &P, int nrhs, const double *xp, double *yn, hipStream_t s) {
    hipEvent_t ev = P.prof.begin(s);
    k_near<NR><<<int(pow8(P.L)), 64, 0, s>>>(P.L, P.leaf_off, P.near_ptr, P.near_s, P.px, P.py,
                                              P.pz, P.cfg.kernel, P.cfg.kernel_param, nrhs, xp,
                                              P.n, yn);
    H3D_LAUNCH_CHECK();
    P.prof.end(s, ev, "near_field", double(P.n) * (32.0 + 8.0 * nrhs),
               double(P.stats.near_pair_evals) * (10.0 + 2.0 * nrhs));
}

}  // namespace

void matvec_run(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                int io_dtype, bool adjoint, hipStream_t s) {
    const int64_t n = P.n;
    if (nrhs > P.scratch_nrhs) {
        P.mem.release(P.xp);
        P.mem.release(P.yp);
        P.mem.release(P.z);
        P.xp = P.mem.alloc_n<double>(n * nrhs);
        P.yp = P.mem.alloc_n<double>(n * nrhs);
        P.z = P.mem.alloc_n<double>(std::max<int64_t>(P.ncols, 1) * nrhs);
        P.scratch_nrhs = nrhs;
    }
    const int io_f32 = io_dtype == H3D_F32;
    {
        hipEvent_t ev = P.prof.begin(s);
        k_gather<<<grid_for(n, 256), 256, 0, s>>>(x, io_f32, ldx, n, int(nrhs), P.perm, P.xp);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "gather", double(n) * (4.0 + (io_f32 ? 4.0 : 8.0) * nrhs + 8.0 * nrhs), 0.0);
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
