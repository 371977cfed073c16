// Products with many right-hand sides on the matrix cores.
//
// With nrhs columns every block apply of Algorithm 2 is a small dense GEMM:
//   near   Y_t += K(t,s) X_s        (m x n) (n x nrhs), K entries evaluated
//                                   on the fly straight into the A operand
//   stage1 Z_b  = V_b^T X_s         (k x n) (n x nrhs)
//   stage2 Y_t += U_b Z_b           (m x k) (k x nrhs), level by level
// (forward products with leaves of at most 16 points on average fuse both
// stages at the finest level: k_leaf_mfma)
// All three run on 16x16x4 MFMA tiles (FP64 MFMA for FP64 factors, FP32 MFMA
// for FP32 and BF16 factors).  Right-hand sides are held point-major (a row of
// NP = 16 ceil(nrhs/16) values per point) so that every B fragment is four
// 64-byte segments.  FP32 tiles are flushed into FP64 registers at least
// every 64 K-steps (the single-tile stage-2 and finest-level kernels after
// every block), so long dot products and the sums over blocks and levels
// carry FP64 accumulation.  Fragment loads are issued from indices clamped
// into the block and masked where the MFMA uses them, so that the loads of
// the next K-steps (or the next block) can be in flight while the current
// MFMAs run.  The adjoint swaps
// U and V and walks the blocks by source box, as in the one-column kernels.
#include "product_items.hpp"

namespace h3d {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// factor loads (global-address loads: the pointers come from block tables)
template <int DT> struct FacB;
template <> struct FacB<H3D_F64> {
    using T = double;
    static __device__ __forceinline__ double ld(const T *p) { return dev::fac_raw<H3D_F64>(p); }
};
template <> struct FacB<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p) { return dev::fac_raw<H3D_F32>(p); }
};
template <> struct FacB<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ float ld(const T *p) {
        return __uint_as_float(uint32_t(dev::fac_raw<H3D_BF16_SCALED>(p)) << 16);
    }
};

// compute type: FP64 factors -> double tiles, otherwise float tiles
template <int DT> struct CT {
    using T = float;
    using V4 = f4;
    static __device__ __forceinline__ V4 mfma(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of the 16x16 output tile held in element j of this lane
    static __device__ __forceinline__ int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};
template <> struct CT<H3D_F64> {
    using T = double;
    using V4 = d4;
    static __device__ __forceinline__ V4 mfma(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int j) { return 4 * j + (lane >> 4); }
};

constexpr int kNT = 4;  // 16-wide RHS tiles per pass (64 columns)

// x (caller order, column-major, io type) -> Xs (sorted, point-major, width NP).
// Through LDS, in caller order: a workgroup takes 64 points
// (consecutive in the caller's order) and 64 right-hand sides, reads the
// columns of x coalesced, and writes each point's 64 values as one
// contiguous piece of its row iperm[i] of Xs.  Columns past nrhs are zero.
template <typename T>
__global__ void __launch_bounds__(256)
    k_gather_t(const void *__restrict__ x, int io_f32, int64_t ldx, int64_t n, int nrhs, int NP,
               const int32_t *__restrict__ iperm, T *__restrict__ Xs) {
    __shared__ T tile[64][65];
    const int64_t i0 = int64_t(blockIdx.x) * 64;
    const int r0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int rr = e >> 6, ii = e & 63;
        const int64_t i = i0 + ii;
        const int r = r0 + rr;
        double v = 0.0;
        if (r < nrhs && i < n)
            v = io_f32 ? double(static_cast<const float *>(x)[r * ldx + i])
                       : static_cast<const double *>(x)[r * ldx + i];
        tile[ii][rr] = T(v);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ii = e >> 6, rr = e & 63;
        const int64_t i = i0 + ii;
        if (i < n && r0 + rr < NP)
            Xs[int64_t(iperm[i]) * NP + r0 + rr] = tile[ii][rr];
    }
}

// Y (sorted, point-major FP64) -> y (caller order, column-major) through LDS:
// a workgroup takes 64 points in the caller's order and 64 right-hand sides,
// reads each point's row iperm[i] of Y contiguously and writes the columns
// of y coalesced.
__global__ void __launch_bounds__(256)
    k_scatter_t(const double *__restrict__ Y, int64_t n, int nrhs, int NP,
                const int32_t *__restrict__ iperm, void *__restrict__ y, int64_t ldy, int io_f32) {
    __shared__ double tile[64][65];
    const int64_t i0 = int64_t(blockIdx.x) * 64;
    const int r0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ii = e >> 6, rr = e & 63;
        const int64_t i = i0 + ii;
        tile[ii][rr] = (i < n && r0 + rr < NP) ? Y[int64_t(iperm[i]) * NP + r0 + rr] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int rr = e >> 6, ii = e & 63;
        const int64_t i = i0 + ii;
        const int r = r0 + rr;
        if (r < nrhs && i < n) {
            if (io_f32)
                static_cast<float *>(y)[r * ldy + i] = float(tile[ii][rr]);
            else
                static_cast<double *>(y)[r * ldy + i] = tile[ii][rr];
        }
    }
}

// caller index -> sorted row
__global__ void k_iperm(int64_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ iperm) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n)
        iperm[perm[p]] = int32_t(p);
}

// ---------------------------------------------------------------------------
// near field: one wave per (leaf, 16-row tile) and pass of kNT RHS tiles
template <int DT>
__global__ void __launch_bounds__(64)
    k_near_mfma(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ leaf_off,
                const int32_t *__restrict__ near_ptr, const int32_t *__restrict__ near_s,
                const double *__restrict__ px, const double *__restrict__ py,
                const double *__restrict__ pz, int kind, double kp,
                const typename CT<DT>::T *__restrict__ Xs, int NP, double *__restrict__ Y) {
    using C = CT<DT>;
    using T = typename C::T;
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int2 it = items[w];
    const int t = it.x;
    const int32_t t0 = leaf_off[t], m = leaf_off[t + 1] - t0;
    const int i = it.y * 16 + (lane & 15);
    const bool ai = i < m;
    const int64_t gi = t0 + (ai ? i : 0);
    const double xi = px[gi], yi = py[gi], zi = pz[gi];
    for (int nb = 0; nb < NP; nb += 16 * kNT) {
        const int ntl = min(kNT, (NP - nb) / 16);
        typename C::V4 acc[kNT];
#pragma unroll
        for (int q = 0; q < kNT; ++q)
            acc[q] = typename C::V4{0, 0, 0, 0};
        for (int e = near_ptr[t]; e < near_ptr[t + 1]; ++e) {
            const int32_t s = near_s[e];
            const int32_t s0 = leaf_off[s], ns = leaf_off[s + 1] - s0;
            constexpr int KU = 1;
            for (int j0 = 0; j0 < ns; j0 += 4 * KU) {
                T a[KU], bv[KU][kNT];
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    const int j = j0 + 4 * u + (lane >> 4);
                    const int64_t gj = s0 + j;
                    a[u] = T(0);
                    if (ai && j < ns && gj != gi) {
                        const double dx = xi - px[gj], dy = yi - py[gj], dz = zi - pz[gj];
                        if (DT == H3D_F64)
                            a[u] = T(dev::kernel_f(kind, kp, sqrt(dx * dx + dy * dy + dz * dz)));
                        else
                            a[u] = T(dev::kernel_f32(kind, float(kp), float(dx * dx + dy * dy + dz * dz)));
                    }
#pragma unroll
                    for (int q = 0; q < kNT; ++q)
                        bv[u][q] = (j < ns && q < ntl) ? Xs[gj * NP + nb + 16 * q + (lane & 15)] : T(0);
                }
#pragma unroll
                for (int u = 0; u < KU; ++u)
#pragma unroll
                    for (int q = 0; q < kNT; ++q)
                        if (q < ntl)
                            acc[q] = C::mfma(a[u], bv[u][q], acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < kNT; ++q)
            if (q < ntl)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = it.y * 16 + C::row(lane, jj);
                    if (r < m)
                        Y[(t0 + r) * int64_t(NP) + nb + 16 * q + (lane & 15)] = double(acc[q][jj]);
                }
    }
}

// ---------------------------------------------------------------------------
// Single-tile forms (one 16-column or 16-row tile per wave; the faster form
// when the level's work items are many and its blocks narrow).
// stage 1: one wave per (block, 16-column tile of its factor)
template <int DT>
__global__ void __launch_bounds__(64)
    k_s1_mfma(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ seg_len,
              const int32_t *__restrict__ seg_off, void *const *__restrict__ seg_ptr,
              const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
              const float *__restrict__ scale2, const typename CT<DT>::T *__restrict__ Xs, int NP,
              typename CT<DT>::T *__restrict__ Z, int panel, const int32_t *__restrict__ leaf_off,
              const int32_t *__restrict__ leaf_of, int shc) {
    using C = CT<DT>;
    using T = typename C::T;
    using F = typename FacB<DT>::T;
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int2 it = items[w];
    const int b = it.x, c0 = it.y * 16;
    const int len = seg_len[b], k = rank[b];
    const int64_t off = seg_off[b], col0 = blk_col0[b];
    const F *__restrict__ p = static_cast<const F *>(seg_ptr[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(scale2[2 * b]) * double(scale2[2 * b + 1]);
    const int ca = c0 + (lane & 15);  // A row (factor column) of this lane
    const bool ac = ca < k;
    for (int nb = 0; nb < NP; nb += 16 * kNT) {
        const int ntl = min(kNT, (NP - nb) / 16);
        typename C::V4 acc[kNT];
        double acc64[kNT][4];
#pragma unroll
        for (int q = 0; q < kNT; ++q) {
            acc[q] = typename C::V4{0, 0, 0, 0};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
                acc64[q][jj] = 0.0;
        }
        if constexpr (DT == H3D_F64) {
            for (int j0 = 0; j0 < len; j0 += 4) {
                const int j = j0 + (lane >> 4);
                const bool aj = j < len;
                int64_t ea = int64_t(ca) * len + j;
                if (panel && ac && aj)  // U_b stored as row panels (adjoint above lc)
                    ea = panel_off(leaf_off, leaf_of, shc, int32_t(off), k, j, ca);
                const T a = (ac && aj) ? T(FacB<DT>::ld(p + ea)) : T(0);
                T bv[kNT];
#pragma unroll
                for (int q = 0; q < kNT; ++q)
                    bv[q] = (aj && q < ntl) ? Xs[(off + j) * NP + nb + 16 * q + (lane & 15)] : T(0);
#pragma unroll
                for (int q = 0; q < kNT; ++q)
                    if (q < ntl)
                        acc[q] = C::mfma(a, bv[q], acc[q]);
            }
        } else {
            // FP32/BF16 tiles (measured: slower with FP64 tiles, whose fragments
            // take twice the registers).  Every load is issued, from a row and
            // column clamped into the block and a tile clamped into the RHS, so
            // that the loads of the next K-step stay countable; the raw values
            // are masked where they are used, and two fragment buffers let the
            // next K-step load while the MFMAs of the current one run (a ring
            // of four K-steps cost a wave per SIMD and was slower).
            const int cc = min(ca, k - 1);
            auto frag = [&](int j0, T &a, T (&bv)[kNT]) {
                const int jc = min(j0 + (lane >> 4), len - 1);
                int64_t ea = int64_t(cc) * len + jc;
                if (panel)  // U_b stored as row panels (adjoint above lc)
                    ea = panel_off(leaf_off, leaf_of, shc, int32_t(off), k, jc, cc);
                a = T(FacB<DT>::ld(p + ea));
#pragma unroll
                for (int q = 0; q < kNT; ++q)
                    bv[q] = Xs[(off + jc) * NP + nb + 16 * min(q, ntl - 1) + (lane & 15)];
            };
            int steps = 0;
            auto step = [&](int j0, const T ar, const T (&br)[kNT]) {
                const bool aj = j0 + (lane >> 4) < len;
                const T a = (ac && aj) ? ar : T(0);
#pragma unroll
                for (int q = 0; q < kNT; ++q)  // rows past the block, tiles past the RHS: 0
                    acc[q] = C::mfma(a, (aj && q < ntl) ? br[q] : T(0), acc[q]);
                if (++steps == 64) {
                    steps = 0;
#pragma unroll
                    for (int q = 0; q < kNT; ++q) {
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj)
                            acc64[q][jj] += double(acc[q][jj]);
                        acc[q] = typename C::V4{0, 0, 0, 0};
                    }
                }
            };
            T a0, b0[kNT], a1, b1[kNT];
            frag(0, a0, b0);
            for (int j0 = 0; j0 < len; j0 += 8) {
                if (j0 + 4 < len)
                    frag(j0 + 4, a1, b1);
                step(j0, a0, b0);
                if (j0 + 4 >= len)
                    break;
                if (j0 + 8 < len)
                    frag(j0 + 8, a0, b0);
                step(j0 + 4, a1, b1);
            }
        }
#pragma unroll
        for (int q = 0; q < kNT; ++q)
            if (q < ntl)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int c = c0 + C::row(lane, jj);
                    if (c < k)
                        Z[(col0 + c) * NP + nb + 16 * q + (lane & 15)] =
                            T((acc64[q][jj] + double(acc[q][jj])) * sc);
                }
    }
}

// stage 1: one wave per (block, 16 MT-column tile of its factor)
template <int DT, int MT>
__global__ void __launch_bounds__(64)
    k_s1_mfma_w(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ seg_len,
                const int32_t *__restrict__ seg_off, void *const *__restrict__ seg_ptr,
                const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
                const float *__restrict__ scale2, const typename CT<DT>::T *__restrict__ Xs, int NP,
                typename CT<DT>::T *__restrict__ Z, int panel, const int32_t *__restrict__ leaf_off,
                const int32_t *__restrict__ leaf_of, int shc, int rows,
                typename CT<DT>::T *__restrict__ Zp) {
    using C = CT<DT>;
    using T = typename C::T;
    using F = typename FacB<DT>::T;
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int2 it = items[w];
    // split columns: item.y = tile + 256 part; the part's partial tile goes to Zp
    const int tile = rows > 0 ? (it.y & 255) : it.y;
    const int b = it.x, c0 = tile * 16 * MT;
    const int len = seg_len[b], k = rank[b];
    int jb = 0, je = len;
    if (rows > 0) {
        jb = min(len, (it.y >> 8) * rows);
        je = min(len, jb + rows);
    }
    const int64_t off = seg_off[b], col0 = blk_col0[b];
    const F *__restrict__ p = static_cast<const F *>(seg_ptr[b]);
    double sc = 1.0;
    if (DT == H3D_BF16_SCALED)
        sc = double(scale2[2 * b]) * double(scale2[2 * b + 1]);
    int ca[MT];
    bool ac[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        ca[t] = c0 + 16 * t + (lane & 15);
        ac[t] = ca[t] < k;
    }
    for (int nb = 0; nb < NP; nb += 16 * kNT) {
        const int ntl = min(kNT, (NP - nb) / 16);
        constexpr int A64 = DT == H3D_F64 ? 1 : MT;
        typename C::V4 acc[MT][kNT];
        double acc64[A64][kNT][4];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int q = 0; q < kNT; ++q)
                acc[t][q] = typename C::V4{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < A64; ++t)
#pragma unroll
            for (int q = 0; q < kNT; ++q)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    acc64[t][q][jj] = 0.0;
        if constexpr (DT == H3D_F64 && MT > 1) {
            for (int j0 = jb; j0 < je; j0 += 4) {
                const int j = j0 + (lane >> 4);
                const bool aj = j < je;
                T a[MT], bv[kNT];
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    int64_t ea = int64_t(ca[t]) * len + j;
                    if (panel && ac[t] && aj)  // U_b stored as row panels (adjoint above lc)
                        ea = panel_off(leaf_off, leaf_of, shc, int32_t(off), k, j, ca[t]);
                    a[t] = (ac[t] && aj) ? T(FacB<DT>::ld(p + ea)) : T(0);
                }
#pragma unroll
                for (int q = 0; q < kNT; ++q)
                    bv[q] = (aj && q < ntl) ? Xs[(off + j) * NP + nb + 16 * q + (lane & 15)] : T(0);
#pragma unroll
                for (int t = 0; t < MT; ++t)
#pragma unroll
                    for (int q = 0; q < kNT; ++q)
                        if (q < ntl)
                            acc[t][q] = C::mfma(a[t], bv[q], acc[t][q]);
            }
        } else if (je > jb && k > 0) {
            // FP32/BF16 tiles, and single FP64 tiles: a ring of D K-steps of
            // fragments in flight.
            // Every load is issued from a row clamped into the item, a column
            // clamped into the block and a tile clamped into the RHS; the raw
            // values are masked where the MFMA uses them, so the sums are
            // those of the plain loop, in the same order.
            constexpr int D = MT >= 4 ? 2 : 4;
            int cc[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t)
                cc[t] = min(ca[t], k - 1);
            auto frag = [&](int j0, T (&a)[MT], T (&bv)[kNT]) {
                const int jc = min(j0 + (lane >> 4), je - 1);
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    int64_t ea = int64_t(cc[t]) * len + jc;
                    if (panel)  // U_b stored as row panels (adjoint above lc)
                        ea = panel_off(leaf_off, leaf_of, shc, int32_t(off), k, jc, cc[t]);
                    a[t] = T(FacB<DT>::ld(p + ea));
                }
#pragma unroll
                for (int q = 0; q < kNT; ++q)
                    bv[q] = Xs[(off + jc) * NP + nb + 16 * min(q, ntl - 1) + (lane & 15)];
            };
            int steps = 0;
            auto step = [&](int j0, const T (&ar)[MT], const T (&br)[kNT]) {
                const bool aj = j0 + (lane >> 4) < je;
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    const T a = (ac[t] && aj) ? ar[t] : T(0);
#pragma unroll
                    for (int q = 0; q < kNT; ++q)  // tiles past the RHS: 0
                        acc[t][q] = C::mfma(a, (aj && q < ntl) ? br[q] : T(0), acc[t][q]);
                }
                if (DT != H3D_F64 && ++steps == 64) {
                    steps = 0;
#pragma unroll
                    for (int t = 0; t < MT; ++t)
#pragma unroll
                        for (int q = 0; q < kNT; ++q) {
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj)
                                acc64[t][q][jj] += double(acc[t][q][jj]);
                            acc[t][q] = typename C::V4{0, 0, 0, 0};
                        }
                }
            };
            T ab[D][MT], bb[D][kNT];
#pragma unroll
            for (int d = 0; d < D; ++d)
                frag(jb + 4 * d, ab[d], bb[d]);
            for (int j0 = jb; j0 < je; j0 += 4 * D) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int js = j0 + 4 * d;
                    if (js < je) {
                        step(js, ab[d], bb[d]);
                        if (js + 4 * D < je)
                            frag(js + 4 * D, ab[d], bb[d]);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int q = 0; q < kNT; ++q)
                if (q < ntl)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int c = c0 + 16 * t + C::row(lane, jj);
                        double v = double(acc[t][q][jj]);
                        if constexpr (DT != H3D_F64)
                            v += acc64[t][q][jj];
                        if (rows > 0)  // every slot of the partial tile, in item order
                            Zp[(w * 16 * MT + 16 * t + C::row(lane, jj)) * int64_t(NP) + nb + 16 * q +
                               (lane & 15)] = T(v * sc);
                        else if (c < k)
                            Z[(col0 + c) * NP + nb + 16 * q + (lane & 15)] = T(v * sc);
                    }
    }
}

// Finest level, forward product: both stages per block in one pass, Z kept on
// chip.  One wave per (target leaf, 16-row tile); for every block of the leaf
// and every 16-column tile of its factors: Z (16 columns x 64 RHS) =
// V_b^T X_s on the matrix cores, handed through wave-private LDS into the B
// layout, then Y_t += U_b Z.  At the leaf level Z (ranks x RHS values) is
// several times the factor bytes, and it never reaches HBM here.  FP32 tiles
// are flushed into FP64 after every block.
template <int DT>
__global__ void __launch_bounds__(64)
    k_leaf_mfma(const int2 *__restrict__ items, int64_t nitems, int64_t gbase,
                const int32_t *__restrict__ leaf_off, const int64_t *__restrict__ grp_begin,
                void *const *__restrict__ uptr, void *const *__restrict__ vptr,
                const int32_t *__restrict__ rank, const int32_t *__restrict__ soff,
                const int32_t *__restrict__ slen, const float *__restrict__ scale2,
                const typename CT<DT>::T *__restrict__ Xs, int NP, double *__restrict__ Y) {
    using C = CT<DT>;
    using T = typename C::T;
    using F = typename FacB<DT>::T;
    __shared__ T zl[16][16 * kNT + 1];  // one Z tile: [column][RHS]
    // metadata of the leaf's next 64 blocks
    __shared__ int32_t s_k[64], s_n[64];
    __shared__ int64_t s_so[64];
    __shared__ const F *s_v[64];
    __shared__ const F *s_u[64];
    __shared__ T s_sc[64];
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int2 it = items[w];
    const int64_t t = it.x;
    const int32_t bs = leaf_off[t], bm = leaf_off[t + 1] - bs;
    const int r0 = it.y * 16;
    const int ia = r0 + (lane & 15);
    const bool ar = ia < bm;
    const int64_t e0 = grp_begin[gbase + t], e1 = grp_begin[gbase + t + 1];
    for (int nb = 0; nb < NP; nb += 16 * kNT) {
        const int ntl = min(kNT, (NP - nb) / 16);
        double acc64[kNT][4];
        typename C::V4 acc[kNT];
#pragma unroll
        for (int q = 0; q < kNT; ++q) {
            acc[q] = typename C::V4{0, 0, 0, 0};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int r = r0 + C::row(lane, jj);
                acc64[q][jj] = (q < ntl && r < bm)
                                   ? Y[(bs + r) * int64_t(NP) + nb + 16 * q + (lane & 15)]
                                   : 0.0;
            }
        }
        // The blocks 64 at a time: their metadata staged in LDS, and (FP32
        // and BF16 fragments) the loads of block i + 1 issued before block
        // i's MFMAs run (two named register sets, used alternately).  The
        // loads are issued for every
        // block, from rows and columns clamped into it (a block of rank 0
        // reads at most 16 entries from its V pointer, which stay inside the
        // padding that follows every chunk of factors), so that the waits for
        // them stay countable; only blocks with k, n <= 16 use the values.
        for (int64_t q0 = e0; q0 < e1; q0 += 64) {
            const int nbk = int(min<int64_t>(64, e1 - q0));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < nbk) {
                const int64_t b = q0 + lane;
                s_k[lane] = rank[b];
                s_n[lane] = slen[b];
                s_so[lane] = soff[b];
                s_v[lane] = static_cast<const F *>(vptr[b]);
                s_u[lane] = static_cast<const F *>(uptr[b]);
                s_sc[lane] = DT == H3D_BF16_SCALED ? T(double(scale2[2 * b]) * double(scale2[2 * b + 1]))
                                                   : T(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            auto load = [&](int i, T (&av)[4], T (&xv)[4][kNT], T (&uv)[4]) {
                const int k = s_k[i], n = s_n[i];
                const int64_t so = s_so[i];
                const F *__restrict__ V = s_v[i];
                // rank 0: both reads go to V, at most 16 entries in
                const F *__restrict__ U = k > 0 ? s_u[i] : V;
                const int cc = min(lane & 15, max(k, 1) - 1);
                const int iu = k > 0 ? min(ia, bm - 1) : min(min(ia, bm - 1), 15);
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int jc = min(4 * st + (lane >> 4), n - 1);
                    av[st] = T(FacB<DT>::ld(V + int64_t(cc) * n + jc));
#pragma unroll
                    for (int q = 0; q < kNT; ++q)
                        xv[st][q] = Xs[(so + jc) * NP + nb + 16 * min(q, ntl - 1) + (lane & 15)];
                    uv[st] = T(FacB<DT>::ld(U + int64_t(min(4 * st + (lane >> 4), max(k, 1) - 1)) * bm + iu));
                }
            };
            auto run = [&](int i, const T (&av)[4], const T (&xv)[4][kNT], const T (&uv)[4]) {
                const int k = s_k[i], n = s_n[i];
                const int64_t so = s_so[i];
                const F *__restrict__ V = s_v[i];
                const F *__restrict__ U = s_u[i];
                const T sc = s_sc[i];
                if (k > 0 && k <= 16 && n <= 16) {
                    // one column tile, at most four K-steps in each stage
                    // (almost every block at this level), loaded in advance
                    typename C::V4 zt[kNT];
#pragma unroll
                    for (int q = 0; q < kNT; ++q)
                        zt[q] = typename C::V4{0, 0, 0, 0};
#pragma unroll
                    for (int st = 0; st < 4; ++st)
                        if (4 * st < n) {
                            const bool aj = 4 * st + (lane >> 4) < n;
                            const T a = ((lane & 15) < k && aj) ? av[st] : T(0);
#pragma unroll
                            for (int q = 0; q < kNT; ++q)
                                zt[q] = C::mfma(a, (aj && q < ntl) ? xv[st][q] : T(0), zt[q]);
                        }
#pragma unroll
                    for (int q = 0; q < kNT; ++q)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj)
                            zl[C::row(lane, jj)][16 * q + (lane & 15)] = zt[q][jj] * sc;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int st = 0; st < 4; ++st)
                        if (4 * st < k) {
                            const int c = 4 * st + (lane >> 4);
                            const bool ak = c < k;
                            const T a = (ar && ak) ? uv[st] : T(0);
#pragma unroll
                            for (int q = 0; q < kNT; ++q)
                                acc[q] = C::mfma(a, (ak && q < ntl) ? zl[c][16 * q + (lane & 15)] : T(0),
                                                 acc[q]);
                        }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                } else {
                    for (int c0 = 0; c0 < k; c0 += 16) {
                        // stage 1: Z tile = V^T X over the source rows
                        const int ca = c0 + (lane & 15);
                        const bool ac = ca < k;
                        typename C::V4 zt[kNT];
#pragma unroll
                        for (int q = 0; q < kNT; ++q)
                            zt[q] = typename C::V4{0, 0, 0, 0};
                        for (int j0 = 0; j0 < n; j0 += 4) {
                            const int j = j0 + (lane >> 4);
                            const bool aj = j < n;
                            const T a = (ac && aj) ? T(FacB<DT>::ld(V + int64_t(ca) * n + j)) : T(0);
#pragma unroll
                            for (int q = 0; q < kNT; ++q) {
                                const T bv = (aj && q < ntl) ? Xs[(so + j) * NP + nb + 16 * q + (lane & 15)]
                                                             : T(0);
                                if (q < ntl)
                                    zt[q] = C::mfma(a, bv, zt[q]);
                            }
                        }
                        // output layout -> [column][RHS] in LDS
#pragma unroll
                        for (int q = 0; q < kNT; ++q)
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj)
                                zl[C::row(lane, jj)][16 * q + (lane & 15)] = zt[q][jj] * sc;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        // stage 2: Y tile += U Z over the tile's columns
                        const int kc = min(16, k - c0);
                        for (int s4 = 0; s4 < kc; s4 += 4) {
                            const int c = s4 + (lane >> 4);
                            const bool ak = c < kc;
                            const T a = (ar && ak) ? T(FacB<DT>::ld(U + int64_t(c0 + c) * bm + ia)) : T(0);
#pragma unroll
                            for (int q = 0; q < kNT; ++q) {
                                const T bv = (ak && q < ntl) ? zl[c][16 * q + (lane & 15)] : T(0);
                                if (q < ntl)
                                    acc[q] = C::mfma(a, bv, acc[q]);
                            }
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    }
                }
                if constexpr (DT != H3D_F64) {
#pragma unroll
                    for (int q = 0; q < kNT; ++q) {
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj)
                            acc64[q][jj] += double(acc[q][jj]);
                        acc[q] = typename C::V4{0, 0, 0, 0};
                    }
                }
            };
            T av0[4], xv0[4][kNT], uv0[4], av1[4], xv1[4][kNT], uv1[4];
            if constexpr (DT == H3D_F64) {
                // FP64 fragments: a second register set costs occupancy
                // (measured slower); each block loads just before it runs
                for (int i = 0; i < nbk; ++i) {
                    load(i, av0, xv0, uv0);
                    run(i, av0, xv0, uv0);
                }
            } else {
                // (past the last block the loads repeat it, unused)
                load(0, av0, xv0, uv0);
                for (int i = 0; i < nbk; i += 2) {
                    load(min(i + 1, nbk - 1), av1, xv1, uv1);
                    run(i, av0, xv0, uv0);
                    if (i + 1 >= nbk)
                        break;
                    load(min(i + 2, nbk - 1), av0, xv0, uv0);
                    run(i + 1, av1, xv1, uv1);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kNT; ++q)
            if (q < ntl)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = r0 + C::row(lane, jj);
                    double v = acc64[q][jj];
                    if constexpr (DT == H3D_F64)
                        v += acc[q][jj];
                    if (r < bm)
                        Y[(bs + r) * int64_t(NP) + nb + 16 * q + (lane & 15)] = v;
                }
    }
}

// split stage-1 columns: Z of every (block, column tile) = its parts' partial
// tiles added in part order; one thread per (group, column, RHS)
template <typename T>
__global__ void k_s1_mfma_reduce(int64_t ngrp, const int32_t *__restrict__ grp,
                                 const int2 *__restrict__ items, int cols,
                                 const int32_t *__restrict__ rank,
                                 const int64_t *__restrict__ blk_col0, const T *__restrict__ Zp,
                                 int NP, T *__restrict__ Z) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(cols) * NP;
    const int64_t g = t / per;
    if (g >= ngrp)
        return;
    const int64_t rem = t - g * per;
    const int u = int(rem / NP), rhs = int(rem - int64_t(u) * NP);
    const int32_t first = grp[2 * g], np = grp[2 * g + 1];
    const int2 it = items[first];
    const int c = (it.y & 255) * cols + u;
    if (c >= rank[it.x])
        return;
    double v = 0.0;
    for (int32_t pp = 0; pp < np; ++pp)
        v += double(Zp[((int64_t(first) + pp) * cols + u) * NP + rhs]);
    Z[(blk_col0[it.x] + c) * int64_t(NP) + rhs] = T(v);
}

// split items of the blocks [b0, b0 + nb): (block, tile + 256 part) with the
// parts of a tile consecutive; one reduction group (first item, parts) per tile
__global__ void k_cnt_split(int64_t b0, int64_t nb, const int32_t *__restrict__ rank,
                            const int32_t *__restrict__ m, const int32_t *__restrict__ n, int cols,
                            int rows, int64_t *__restrict__ cnt, int64_t *__restrict__ gcnt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nb)
        return;
    const int64_t b = b0 + i;
    const int nt = (rank[b] + cols - 1) / cols;
    const int np = max(1, (max(m[b], n[b]) + rows - 1) / rows);
    cnt[i] = int64_t(nt) * np;
    gcnt[i] = nt;
}

__global__ void k_fill_split(int64_t b0, int64_t nb, const int32_t *__restrict__ rank,
                             const int32_t *__restrict__ m, const int32_t *__restrict__ n, int cols,
                             int rows, const int64_t *__restrict__ off,
                             const int64_t *__restrict__ goff, int32_t *__restrict__ items,
                             int32_t *__restrict__ grp) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nb)
        return;
    const int64_t b = b0 + i;
    const int nt = (rank[b] + cols - 1) / cols;
    const int np = max(1, (max(m[b], n[b]) + rows - 1) / rows);
    for (int t = 0; t < nt; ++t) {
        const int64_t f = off[i] + int64_t(t) * np;
        grp[2 * (goff[i] + t)] = int32_t(f);
        grp[2 * (goff[i] + t) + 1] = np;
        for (int pp = 0; pp < np; ++pp) {
            items[2 * (f + pp)] = int32_t(b);
            items[2 * (f + pp) + 1] = t + 256 * pp;
        }
    }
}

// ---------------------------------------------------------------------------
// work items: (leaf, row tile), (block, column tile), (box, row tile)
__global__ void k_cnt_rowtiles(int64_t nb, int sh, const int32_t *__restrict__ leaf_off,
                               int tile, int64_t *__restrict__ cnt) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b < nb)
        cnt[b] = (leaf_off[(b + 1) << sh] - leaf_off[b << sh] + tile - 1) / tile;
}

__global__ void k_fill_tiles(int64_t nb, const int64_t *__restrict__ cnt_scan,
                             const int64_t *__restrict__ cnt_raw, int64_t id0,
                             int32_t *__restrict__ items) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb)
        return;
    const int64_t o = cnt_scan[b];
    for (int64_t q = 0; q < cnt_raw[b]; ++q) {
        items[2 * (o + q)] = int32_t(id0 + b);
        items[2 * (o + q) + 1] = int32_t(q);
    }
}

__global__ void k_cnt_coltiles(int64_t b0, int64_t nb, const int32_t *__restrict__ rank,
                               int tile, int64_t *__restrict__ cnt) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b < nb)
        cnt[b] = (rank[b0 + b] + tile - 1) / tile;
}

// tile counts of the blocks at positions b0 .. b0 + nb of perm (or of the
// level order when perm is null)
__global__ void k_cnt_coltiles_perm(int64_t b0, int64_t nb, const int32_t *__restrict__ rank,
                                    const int64_t *__restrict__ perm, int tile,
                                    int64_t *__restrict__ cnt) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b < nb)
        cnt[b] = (rank[perm ? perm[b0 + b] : b0 + b] + tile - 1) / tile;
}

// items made over positions of perm: replaces each position by its block
__global__ void k_items_perm(int64_t n, const int64_t *__restrict__ perm,
                             int32_t *__restrict__ items) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        items[2 * i] = int32_t(perm[items[2 * i]]);
}

// builds items for nb consecutive units whose tile counts are in cnt[0..nb)
int32_t *make_items(Plan &P, int64_t nb, int64_t id0, int64_t *cnt, int64_t *count, hipStream_t s) {
    int64_t *raw = P.mem.alloc_n<int64_t>(nb + 1);
    H3D_HIP(hipMemcpyAsync(raw, cnt, sizeof(int64_t) * size_t(nb), hipMemcpyDeviceToDevice, s));
    H3D_HIP(hipMemsetAsync(cnt + nb, 0, sizeof(int64_t), s));
    const int64_t tot = scan_exclusive_i64(P, cnt, cnt, nb + 1, s);
    int32_t *items = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(tot, 1));
    k_fill_tiles<<<grid_for(nb, 256), 256, 0, s>>>(nb, cnt, raw, id0, items);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipStreamSynchronize(s));
    P.mem.release(raw);
    *count = tot;
    return items;
}

// 16-column tiles per stage-1 wave (by the level's mean rank) and 16-row
// tiles per stage-2 wave (by the level's mean box size)
// (measured: wider tiles pay off for FP64 tiles only; FP32 tiles carry FP64
// flush registers as well and lose more to occupancy than they gain)
int tiles_for(int v, int dt) {
    if (dt != H3D_F64)
        return 1;
    return v >= 48 ? 4 : (v >= 24 ? 2 : 1);
}

// Levels whose columns would be split take the ring kernel instead
// when it has at least this many items (four per SIMD)
constexpr int64_t kRingMinItems = 4096;

// stage-1 columns of boxes above this size are split into parts of this many rows
constexpr int kMfmaSplitBox = 2048;
constexpr int kMfmaSplitRows = 1024;

void ensure_batched_tables(Plan &P, hipStream_t s) {
    if (P.bt_ready)
        return;
    const int L = P.L;
    for (int l = 1; l <= L; ++l) {
        const int64_t nbl = P.lvl_blk[l + 1] - P.lvl_blk[l];
        const int mean_rank = nbl > 0 ? int(P.lvl_rank_sum[l] / nbl) : 0;
        // (split items keep the tile index in 8 bits)
        P.bt_split[l] =
            (P.mean_box[l] > kMfmaSplitBox && P.stats.rank_max < 255 * 16) ? kMfmaSplitRows : 0;
        // wide stage-1 tiles for wide blocks only, where they still leave
        // enough waves (measured: four tiles help at mean rank >= 48, two do not)
        const int t1 = tiles_for(mean_rank, P.factor_dtype) == 4 ? 4 : 1;
        P.bt_mt1[l] = (P.bt_split[l] == 0 && nbl * ((mean_rank + 16 * t1 - 1) / (16 * t1)) >= 8192)
                          ? t1 : 1;
    }
    // near: (leaf, row tile)
    {
        const int64_t nl = pow8(L);
        int64_t *cnt = P.mem.alloc_n<int64_t>(nl + 1);
        k_cnt_rowtiles<<<grid_for(nl, 256), 256, 0, s>>>(nl, 0, P.leaf_off, 16, cnt);
        H3D_LAUNCH_CHECK();
        P.bt_near = make_items(P, nl, 0, cnt, &P.bt_nnear, s);
        P.mem.release(cnt);
    }
    for (int l = 1; l <= L; ++l) {
        // stage 1: (block, column tile)
        const int64_t b0 = P.lvl_blk[l], nb = P.lvl_blk[l + 1] - b0;
        P.bt_s1[l] = nullptr;
        P.bt_ns1[l] = 0;
        if (nb > 0 && P.bt_split[l] > 0) {
            const int cols = 16 * P.bt_mt1[l];
            int64_t *cnt = P.mem.alloc_n<int64_t>(nb + 1);
            int64_t *gcnt = P.mem.alloc_n<int64_t>(nb + 1);
            H3D_HIP(hipMemsetAsync(cnt + nb, 0, sizeof(int64_t), s));
            H3D_HIP(hipMemsetAsync(gcnt + nb, 0, sizeof(int64_t), s));
            k_cnt_split<<<grid_for(nb, 256), 256, 0, s>>>(b0, nb, P.blk_rank, P.blk_m, P.blk_n,
                                                          cols, P.bt_split[l], cnt, gcnt);
            H3D_LAUNCH_CHECK();
            const int64_t ni = scan_exclusive_i64(P, cnt, cnt, nb + 1, s);
            const int64_t ng = scan_exclusive_i64(P, gcnt, gcnt, nb + 1, s);
            int32_t *items = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(ni, 1));
            int32_t *grp = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(ng, 1));
            k_fill_split<<<grid_for(nb, 256), 256, 0, s>>>(b0, nb, P.blk_rank, P.blk_m, P.blk_n,
                                                           cols, P.bt_split[l], cnt, gcnt, items,
                                                           grp);
            H3D_LAUNCH_CHECK();
            H3D_HIP(hipStreamSynchronize(s));
            P.mem.release(cnt);
            P.mem.release(gcnt);
            P.bt_s1[l] = items;
            P.bt_ns1[l] = ni;
            P.bt_grp[l] = grp;
            P.bt_ngrp[l] = ng;
        } else if (nb > 0) {
            int64_t *cnt = P.mem.alloc_n<int64_t>(nb + 1);
            k_cnt_coltiles<<<grid_for(nb, 256), 256, 0, s>>>(b0, nb, P.blk_rank,
                                                            16 * P.bt_mt1[l], cnt);
            H3D_LAUNCH_CHECK();
            P.bt_s1[l] = make_items(P, nb, b0, cnt, &P.bt_ns1[l], s);
            P.mem.release(cnt);
        }
        if (nb > 0) {
            // the ring kernels' items: (block, 16 MT columns), blocks in level
            // order (grouped by target box: the adjoint's rows of X) and in
            // source order (the forward's); FP64 tiles two columns wide
            const int cols = P.factor_dtype == H3D_F64 ? 32 : 16 * s1_ring_tiles(P, l);
            for (int dir = 0; dir < 2; ++dir) {
                const int64_t *perm = dir == 0 ? P.src_blk : nullptr;
                int64_t *cnt4 = P.mem.alloc_n<int64_t>(nb + 1);
                k_cnt_coltiles_perm<<<grid_for(nb, 256), 256, 0, s>>>(b0, nb, P.blk_rank, perm,
                                                                     cols, cnt4);
                H3D_LAUNCH_CHECK();
                int64_t cnt_items = 0;
                int32_t *items = make_items(P, nb, b0, cnt4, &cnt_items, s);
                P.mem.release(cnt4);
                if (perm && cnt_items > 0) {
                    k_items_perm<<<grid_for(cnt_items, 256), 256, 0, s>>>(cnt_items, perm, items);
                    H3D_LAUNCH_CHECK();
                }
                P.bt_s1r[l][dir] = items;
                P.bt_ns1r[l][dir] = cnt_items;
            }
        }
        // stage 2: (box, 64-row tile) for the boxes of level l
        const int64_t nbox = pow8(l);
        {
            int64_t *cnt4 = P.mem.alloc_n<int64_t>(nbox + 1);
            k_cnt_rowtiles<<<grid_for(nbox, 256), 256, 0, s>>>(nbox, 3 * (L - l), P.leaf_off, 64,
                                                              cnt4);
            H3D_LAUNCH_CHECK();
            P.bt_s2r[l] = make_items(P, nbox, 0, cnt4, &P.bt_ns2r[l], s);
            P.mem.release(cnt4);
            P.bt_s2k[l][0] = s2_ring_steps(P, l, false, s);
            P.bt_s2k[l][1] = s2_ring_steps(P, l, true, s);
            if (P.factor_dtype == H3D_BF16_SCALED)
                P.bt_s2k16[l] = s2_bf16_steps(P, l, s);
            if (l < P.chunk_level)
                P.bt_pk[l] = panel_steps(P, l, s);
        }
    }
    P.iperm = P.mem.alloc_n<int32_t>(std::max<int64_t>(P.n, 1));
    k_iperm<<<grid_for(P.n, 256), 256, 0, s>>>(P.n, P.perm, P.iperm);
    H3D_LAUNCH_CHECK();
    P.bt_ready = true;
}

template <int DT>
void batched_dt(Plan &P, const void *x, void *y, int nrhs, int64_t ldx, int64_t ldy, int io_f32,
                bool adjoint, hipStream_t s) {
    using T = typename CT<DT>::T;
    const int64_t n = P.n;
    const int NP = 16 * ((nrhs + 15) / 16);
    const size_t need_x = size_t(n) * NP * sizeof(T);
    const size_t need_y = size_t(n) * NP * sizeof(double);
    const size_t need_z = size_t(std::max<int64_t>(P.ncols, 1)) * NP * sizeof(T);
    ensure_batched_tables(P, s);
    // partial tiles of the split stage-1 levels (sized for both directions)
    size_t need_zp = 0;
    for (int l = 1; l <= P.L; ++l)
        if (P.bt_split[l] > 0 && P.bt_ns1[l] > 0)
            need_zp = std::max(need_zp, size_t(P.bt_ns1[l]) * 16 * P.bt_mt1[l] * NP * sizeof(T));
    // forward products with BF16 factors run the far field on the BF16 matrix
    // cores, with x split into BF16 hi/lo words
    const bool bf16mc = DT == H3D_BF16_SCALED && !adjoint;
    const size_t need_xh = bf16mc ? size_t(n) * NP * sizeof(uint32_t) : 0;
    // every buffer is grown before the first launch of the product
    if (need_x > P.bx_bytes || need_y > P.by_bytes || need_z > P.bz_bytes ||
        need_zp > P.bzp_bytes || need_xh > P.bxh_bytes) {
        if (P.bx || P.bzp || P.bxh)
            before_release(P, "a product with more right-hand sides");
        if (need_xh > P.bxh_bytes) {
            P.mem.release(P.bxh);
            P.bxh = nullptr;
            P.bxh_bytes = 0;
            P.bxh = P.mem.alloc(need_xh);
            P.bxh_bytes = need_xh;
        }
        if (need_x > P.bx_bytes || need_y > P.by_bytes || need_z > P.bz_bytes) {
            P.mem.release(P.bx);
            P.mem.release(P.by);
            P.mem.release(P.bz);
            P.bx = P.by = P.bz = nullptr;
            P.bx_bytes = P.by_bytes = P.bz_bytes = 0;
            P.bx = P.mem.alloc(need_x);
            P.by = P.mem.alloc(need_y);
            P.bz = P.mem.alloc(need_z);
            P.bx_bytes = need_x;
            P.by_bytes = need_y;
            P.bz_bytes = need_z;
        }
        if (need_zp > P.bzp_bytes) {
            P.mem.release(P.bzp);
            P.bzp = nullptr;
            P.bzp_bytes = 0;
            P.bzp = P.mem.alloc(need_zp);
            P.bzp_bytes = need_zp;
        }
    }
    T *Xs = static_cast<T *>(P.bx);
    double *Y = static_cast<double *>(P.by);
    T *Z = static_cast<T *>(P.bz);
    const double es = DT == H3D_F64 ? 8.0 : (DT == H3D_F32 ? 4.0 : 2.0);
    {
        hipEvent_t ev = P.prof.begin(s);
        const dim3 grid(unsigned((n + 63) / 64), unsigned(NP / 64 + (NP % 64 ? 1 : 0)));
        k_gather_t<T><<<grid, 256, 0, s>>>(x, io_f32, ldx, n, nrhs, NP, P.iperm, Xs);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "k_gather_pm", double(n) * (4.0 + (io_f32 ? 4 : 8) * nrhs + sizeof(T) * NP), 0.0);
    }
    // a level's far field runs on the BF16 matrix cores when its stage-1
    // items fill the GPU (the few long columns of the coarsest levels take
    // the FP32 row-split kernels; a level's z is written and read in one form)
    auto bf16_level = [&](int l) { return P.bt_ns1r[l][0] >= kRingMinItems; };
    uint32_t *Xh = static_cast<uint32_t *>(P.bxh);
    uint32_t *Zh = reinterpret_cast<uint32_t *>(P.bz);
    if (bf16mc) {
        hipEvent_t ev = P.prof.begin(s);
        launch_split_x(reinterpret_cast<const float *>(Xs), n * NP, Xh, s);
        P.prof.end(s, ev, "k_split_x", double(n) * NP * 8.0, 0.0);
    }
    {
        hipEvent_t ev = P.prof.begin(s);
        // FP32 entries: one wave per leaf when every leaf holds at most 64
        // rows, one per (leaf, 16-row tile) otherwise and for FP64 entries
        const bool by_leaf = DT != H3D_F64 && P.bt_nnear > 0 &&
                             launch_near_leaves(P, reinterpret_cast<const float *>(Xs), NP, Y, s);
        if (P.bt_nnear > 0 && !by_leaf)
            k_near_mfma<DT><<<int(P.bt_nnear), 64, 0, s>>>(
                reinterpret_cast<const int2 *>(P.bt_near), P.bt_nnear, P.leaf_off, P.near_ptr,
                P.near_s, P.px, P.py, P.pz, P.cfg.kernel, P.cfg.kernel_param, Xs, NP, Y);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "k_near_mfma", double(n) * (32.0 + 16.0 * NP),
                   double(P.stats.near_pair_evals) * (10.0 + 2.0 * NP));
    }
    // forward products with small leaves run both stages of the finest level
    // in k_leaf_mfma.  Measured on 262,144 points (leaves of 8): FP32 3.7 ms
    // fused against 6.0 ms in two launches, FP64 5.7 against 8.1; with leaves
    // of about 32 points (1,048,576 points) the fused chain was slower (62
    // against 27 ms, FP32)
    const int lfuse = (adjoint || P.mean_box[P.L] > kLeafRows) ? 0 : P.L;
    // larger leaves (FP32/BF16 factors): both stages per leaf with z kept in
    // registers (k_leaf_fused)
    const int lfused = (DT != H3D_F64 && lfuse == 0 && P.L >= 1 && leaf_fused_tables(P, s))
                           ? P.L
                           : 0;
    for (int l = 1; l <= P.L; ++l) {
        if (P.bt_ns1[l] == 0 || l == lfuse || l == lfused)
            continue;
        hipEvent_t ev = P.prof.begin(s);
        // split levels: partial tiles of every row part, then their sum
        T *Zp = P.bt_split[l] > 0 ? static_cast<T *>(P.bzp) : nullptr;
#define H3D_S1M(MT)                                                                         \
    k_s1_mfma_w<DT, MT><<<int(P.bt_ns1[l]), 64, 0, s>>>(                                    \
        reinterpret_cast<const int2 *>(P.bt_s1[l]), P.bt_ns1[l], adjoint ? P.blk_m : P.blk_n, \
        adjoint ? P.blk_toff : P.blk_soff, adjoint ? P.blk_uptr : P.blk_vptr, P.blk_rank,     \
        P.blk_col0, P.blk_scale, Xs, NP, Z, int(adjoint && l < P.chunk_level), P.leaf_off,    \
        P.leaf_of, 3 * (P.L - P.chunk_level), P.bt_split[l], Zp)
        // the ring kernel wherever its items fill the GPU; the few long
        // columns of the coarsest levels keep the row-split kernels
        const int dir = adjoint ? 1 : 0;
        const bool ring = P.bt_split[l] == 0 || P.bt_ns1r[l][dir] >= kRingMinItems;
        if (DT == H3D_F64 && ring)
            launch_s1_ring64(P, l, adjoint, reinterpret_cast<const int2 *>(P.bt_s1r[l][dir]),
                             P.bt_ns1r[l][dir], reinterpret_cast<const double *>(Xs), NP,
                             reinterpret_cast<double *>(Z), s);
        else if (bf16mc && bf16_level(l))
            launch_s1_bf16(P, l, reinterpret_cast<const int2 *>(P.bt_s1r[l][0]), P.bt_ns1r[l][0], Xh,
                           NP, Zh, s);
        else if (ring)
            launch_s1_ring(P, l, adjoint, reinterpret_cast<const int2 *>(P.bt_s1r[l][dir]),
                           P.bt_ns1r[l][dir], reinterpret_cast<const float *>(Xs), NP,
                           reinterpret_cast<float *>(Z), s);
        else if (P.bt_mt1[l] == 4)
            H3D_S1M(4);
        else if (P.bt_mt1[l] == 2)
            H3D_S1M(2);
        else if (P.bt_split[l] > 0)
            H3D_S1M(1);
        else
            k_s1_mfma<DT><<<int(P.bt_ns1[l]), 64, 0, s>>>(
                reinterpret_cast<const int2 *>(P.bt_s1[l]), P.bt_ns1[l],
                adjoint ? P.blk_m : P.blk_n, adjoint ? P.blk_toff : P.blk_soff,
                adjoint ? P.blk_uptr : P.blk_vptr, P.blk_rank, P.blk_col0, P.blk_scale, Xs, NP, Z,
                int(adjoint && l < P.chunk_level), P.leaf_off, P.leaf_of,
                3 * (P.L - P.chunk_level));
#undef H3D_S1M
        if (!(bf16mc && bf16_level(l)) && !ring && P.bt_split[l] > 0) {
            H3D_LAUNCH_CHECK();
            const int cols = 16 * P.bt_mt1[l];
            const int64_t nt = P.bt_ngrp[l] * cols * NP;
            k_s1_mfma_reduce<T><<<grid_for(nt, 256), 256, 0, s>>>(
                P.bt_ngrp[l], P.bt_grp[l], reinterpret_cast<const int2 *>(P.bt_s1[l]), cols,
                P.blk_rank, P.blk_col0, Zp, NP, Z);
        }
        H3D_LAUNCH_CHECK();
        const double ent = double(adjoint ? P.lvl_entries_u[l] : P.lvl_entries_v[l]);
        char name[48];
        if (bf16mc && bf16_level(l))
            snprintf(name, sizeof(name), P.prof.levels ? "k_s1_bf16_L%d" : "k_s1_bf16", l);
        else
            snprintf(name, sizeof(name), P.prof.levels ? "k_s1_mfma_L%d" : "k_s1_mfma", l);
        P.prof.end(s, ev, name, ent * es + double(P.lvl_rank_sum[l]) * sizeof(T) * NP,
                   2.0 * ent * NP);
    }
    for (int l = 1; l <= P.L; ++l) {
        if (P.bt_ns2r[l] == 0 || P.lvl_blk[l + 1] <= P.lvl_blk[l] || l == lfuse || l == lfused)
            continue;
        hipEvent_t ev = P.prof.begin(s);
        if constexpr (DT != H3D_F64) {
            if (bf16mc && bf16_level(l))
                launch_s2_bf16(P, l, reinterpret_cast<const int2 *>(P.bt_s2r[l]), P.bt_ns2r[l], Zh,
                               NP, Y, s);
            else
                launch_s2_ring(P, l, adjoint, reinterpret_cast<const int2 *>(P.bt_s2r[l]),
                               P.bt_ns2r[l], reinterpret_cast<const float *>(Z), NP, Y, s);
        } else {
            launch_s2_ring64(P, l, adjoint, reinterpret_cast<const int2 *>(P.bt_s2r[l]),
                             P.bt_ns2r[l], reinterpret_cast<const double *>(Z), NP, Y, s);
        }
        H3D_LAUNCH_CHECK();
        const double ent = double(adjoint ? P.lvl_entries_v[l] : P.lvl_entries_u[l]);
        char name2[48];
        if (bf16mc && bf16_level(l))
            snprintf(name2, sizeof(name2), P.prof.levels ? "k_s2_bf16_L%d" : "k_s2_bf16", l);
        else
            snprintf(name2, sizeof(name2), P.prof.levels ? "k_s2_mfma_L%d" : "k_s2_mfma", l);
        P.prof.end(s, ev, name2,
                   ent * es + double(P.lvl_rank_sum[l]) * sizeof(T) * NP + double(n) * 16.0 * NP,
                   2.0 * ent * NP);
    }
    if (lfuse >= 1 && P.lvl_blk[lfuse + 1] > P.lvl_blk[lfuse] && P.bt_nnear > 0) {
        const int l = lfuse;
        hipEvent_t ev = P.prof.begin(s);
        k_leaf_mfma<DT><<<int(P.bt_nnear), 64, 0, s>>>(
            reinterpret_cast<const int2 *>(P.bt_near), P.bt_nnear, P.box_base[l], P.leaf_off,
            P.tgt_begin, P.blk_uptr, P.blk_vptr, P.blk_rank, P.blk_soff, P.blk_n, P.blk_scale, Xs,
            NP, Y);
        H3D_LAUNCH_CHECK();
        const double ent = double(P.lvl_entries_u[l] + P.lvl_entries_v[l]);
        char name[48];
        snprintf(name, sizeof(name), P.prof.levels ? "k_leaf_mfma_L%d" : "k_leaf_mfma", l);
        P.prof.end(s, ev, name, ent * es + double(n) * 16.0 * NP, 4.0 * ent * NP / 2.0);
    }
    if constexpr (DT != H3D_F64) {
        if (lfused >= 1 && P.lvl_blk[lfused + 1] > P.lvl_blk[lfused]) {
            const int l = lfused;
            hipEvent_t ev = P.prof.begin(s);
            launch_leaf_fused(P, reinterpret_cast<const float *>(Xs), NP, Y, adjoint, s);
            const double ent = double(P.lvl_entries_u[l] + P.lvl_entries_v[l]);
            char name[48];
            snprintf(name, sizeof(name), P.prof.levels ? "k_leaf_fused_L%d" : "k_leaf_fused", l);
            P.prof.end(s, ev, name, ent * es + double(n) * 16.0 * NP, 2.0 * ent * NP);
        }
    }
    {
        hipEvent_t ev = P.prof.begin(s);
        const dim3 grid(unsigned((n + 63) / 64), unsigned(NP / 64 + (NP % 64 ? 1 : 0)));
        k_scatter_t<<<grid, 256, 0, s>>>(Y, n, nrhs, NP, P.iperm, y, ldy, io_f32);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "k_scatter_pm", double(n) * (4.0 + 8.0 * nrhs + (io_f32 ? 4 : 8) * nrhs), 0.0);
    }
}

}  // namespace

void matvec_batched(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                    int io_dtype, bool adjoint, hipStream_t s) {
    const int io_f32 = io_dtype == H3D_F32;
    switch (P.factor_dtype) {
    case H3D_F64:
        batched_dt<H3D_F64>(P, x, y, int(nrhs), ldx, ldy, io_f32, adjoint, s);
        break;
    case H3D_F32:
        batched_dt<H3D_F32>(P, x, y, int(nrhs), ldx, ldy, io_f32, adjoint, s);
        break;
    default:
        batched_dt<H3D_BF16_SCALED>(P, x, y, int(nrhs), ldx, ldy, io_f32, adjoint, s);
        break;
    }
}

}  // namespace h3d
