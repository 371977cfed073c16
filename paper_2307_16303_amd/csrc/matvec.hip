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
// stage 1: z[col] = dot(column col of its block's factor, x segment).
// Work item = (block, first column); a wave streams up to `span` columns of
// the block, NS = 64/S columns side by side (S lanes per column) and U such
// groups per pass, so every lane keeps U independent loads in flight.
struct S1Level {
    int64_t i0, i1;  // items of this level
    int S;           // lanes per column
    int span;        // columns per item
};
struct S1Tab {
    S1Level lv[kMaxLevels + 1];
    int nlev;
};

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

template <int S, int DT, int NR>
__device__ __forceinline__ void stage1_item(int2 item, int span, const int64_t *__restrict__ blk_col0,
                                            const int32_t *__restrict__ rank,
                                            const int32_t *__restrict__ seg_len,
                                            const int32_t *__restrict__ seg_off,
                                            void *const *__restrict__ seg_ptr,
                                            const float *__restrict__ scale2, int nrhs,
                                            const double *__restrict__ xp, int64_t n,
                                            double *__restrict__ z, int64_t ldz) {
    using T = typename Fac<DT>::T;
    constexpr int NS = 64 / S;
    constexpr int U = S >= 32 ? 8 : 4;
    const int lane = threadIdx.x & 63;
    const int r = lane % S, sub = lane / S;
    const int b = item.x;
    const int len = seg_len[b];
    const int64_t off = seg_off[b];
    const int64_t col0 = blk_col0[b];
    const int k = rank[b];
    const T *p = static_cast<const T *>(seg_ptr[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(scale2[2 * b]) * double(scale2[2 * b + 1]);
    const int cend = min(item.y + span, k);
    for (int rb = 0; rb < nrhs; rb += NR) {
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
                    xv[q] = (NR == 1 || rb + q < nrhs) ? xp[(rb + q) * n + off + j] : 0.0;
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = cb + sub + u * NS;
                    v[u] = c < cend ? Fac<DT>::ld(p + int64_t(c) * len + j) : 0.0;
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
                            if (NR == 1 || rb + q < nrhs)
                                z[(rb + q) * ldz + col0 + c] = acc[u][q] * sc;
                }
            }
        }
    }
}

template <int DT, int NR>
__global__ void __launch_bounds__(256)
    k_stage1(S1Tab tab, int64_t nitems, const int2 *__restrict__ items,
             const int64_t *__restrict__ blk_col0, const int32_t *__restrict__ rank,
             const int32_t *__restrict__ seg_len, const int32_t *__restrict__ seg_off,
             void *const *__restrict__ seg_ptr, const float *__restrict__ scale2, int nrhs,
             const double *__restrict__ xp, int64_t n, double *__restrict__ z, int64_t ldz) {
    const int64_t w = uniform64((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
    if (w >= nitems)
        return;
    int li = 0;
    while (li + 1 < tab.nlev && w >= tab.lv[li + 1].i0)
        ++li;
    const int S = tab.lv[li].S, span = tab.lv[li].span;
    const int2 it = items[w];
    switch (S) {
    case 4:
        stage1_item<4, DT, NR>(it, span, blk_col0, rank, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    case 8:
        stage1_item<8, DT, NR>(it, span, blk_col0, rank, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    case 16:
        stage1_item<16, DT, NR>(it, span, blk_col0, rank, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    case 32:
        stage1_item<32, DT, NR>(it, span, blk_col0, rank, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    default:
        stage1_item<64, DT, NR>(it, span, blk_col0, rank, seg_len, seg_off, seg_ptr, scale2, nrhs, xp, n, z, ldz);
        break;
    }
}

// ---------------------------------------------------------------------------
// stage 2: one wave per box of the chunk level, one lane per row.  At levels
// up to the chunk level every lane of the wave lies in the same box, so the
// block metadata and z are wave-uniform (scalar loads) and each lane streams
// one column slice of U per load, U2 loads in flight.
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
            v[u] = Fac<DT>::ld(p + int64_t(c + u) * bm);
#pragma unroll
        for (int u = 0; u < U2; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (NR == 1 || rb + q < nrhs)
                    acc[q] += v[u] * zz[(rb + q) * ldz + c + u];
    }
    for (; c < k; ++c) {
        const double v = Fac<DT>::ld(p + int64_t(c) * bm);
#pragma unroll
        for (int q = 0; q < NR; ++q)
            if (NR == 1 || rb + q < nrhs)
                acc[q] += v * zz[(rb + q) * ldz + c];
    }
}

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
    const int64_t B = uniform64((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
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
            // levels whose boxes contain the whole chunk box: wave-uniform
            for (int l = 1; l <= lc; ++l) {
                const int sh = 3 * (L - l);
                const int64_t t = B >> (3 * (lc - l));
                const int64_t g = tab.box_base[l] + t;
                const int32_t bs = leaf_off[t << sh];
                const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                const int32_t loc = rr - bs;
                const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                for (int64_t e = e0; e < e1; ++e) {
                    const int64_t bi = grp_blk ? grp_blk[e] : e;
                    const T *p = static_cast<const T *>(fptr[bi]) + loc;
                    stage2_block<DT, NR, 8>(p, bm, rank[bi], z + blk_col0[bi], ldz, rb, nrhs, acc);
                }
            }
            // finer levels: every lane follows the box of its own row
            for (int l = lc + 1; l <= L; ++l) {
                const int sh = 3 * (L - l);
                const int64_t t = int64_t(leaf) >> sh;
                const int64_t g = tab.box_base[l] + t;
                const int32_t bs = leaf_off[t << sh];
                const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                const int32_t loc = rr - bs;
                const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                for (int64_t e = e0; e < e1; ++e) {
                    const int64_t bi = grp_blk ? grp_blk[e] : e;
                    const T *p = static_cast<const T *>(fptr[bi]) + loc;
                    stage2_block<DT, NR, 4>(p, bm, rank[bi], z + blk_col0[bi], ldz, rb, nrhs, acc);
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

template <int DT, int NR>
void launch_far(Plan &P, bool adjoint, int nrhs, const double *xp, double *z, const double *yn,
                void *y, int64_t ldy, int io_f32, hipStream_t s) {
    const int64_t n = P.n;
    const int L = P.L;
    const size_t es = DT == H3D_F64 ? 8 : (DT == H3D_F32 ? 4 : 2);
    // stage 1
    if (P.nitems > 0) {
        S1Tab tab{};
        int nl = 0;
        for (int l = 1; l <= L; ++l) {
            S1Level lv;
            lv.i0 = P.lvl_item[l];
            lv.i1 = P.lvl_item[l + 1];
            lv.S = P.s1_width[l];
            lv.span = P.s1_span[l];
            tab.lv[nl++] = lv;
        }
        tab.nlev = nl;
        hipEvent_t ev = P.prof.begin(s);
        const int32_t *len = adjoint ? P.blk_m : P.blk_n;
        const int32_t *off = adjoint ? P.blk_toff : P.blk_soff;
        void *const *ptr = adjoint ? P.blk_uptr : P.blk_vptr;
        k_stage1<DT, NR><<<grid_for(P.nitems * 64, 256), 256, 0, s>>>(
            tab, P.nitems, reinterpret_cast<const int2 *>(P.items), P.blk_col0, P.blk_rank, len,
            off, ptr, P.blk_scale, nrhs, xp, n, z, P.ncols);
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
        S2Tab tab{};
        for (int l = 0; l <= kMaxLevels; ++l)
            tab.box_base[l] = P.box_base[l];
        tab.L = L;
        tab.lc = P.chunk_level;
        hipEvent_t ev = P.prof.begin(s);
        const int64_t nchunk = pow8(P.chunk_level);
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
