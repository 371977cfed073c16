// Many right-hand sides, FP32/BF16 factors: stage 1 of one level, Z_b = V_b^T
// X_s (forward; the adjoint reads U_b and the target rows), with a deep ring
// of fragment loads.
//
// One wave per (block, 16 MT factor columns): MT 16-column tiles against the
// four 16-column right-hand-side tiles, 4 MT FP32 MFMAs per K-step of four
// source rows, so every X fragment feeds MT MFMAs and every factor fragment
// four.  The fragments of the next D K-steps are in flight while a step's
// MFMAs run.  Every load is issued from a row and column clamped into the
// block and masked where the MFMA uses it.  Levels whose boxes hold at most
// 256 points sum each column's rows in FP32 (at most 64 K-steps, as the other
// many-RHS kernels flush); longer ones flush the FP32 tiles into FP64 sums
// every 64 K-steps.  Levels split into row parts keep the split kernels.
#include "product_items.hpp"

namespace h3d {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int DT> struct SFac;
template <> struct SFac<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p) { return dev::fac_raw<H3D_F32>(p); }
};
template <> struct SFac<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ float ld(const T *p) {
        return __uint_as_float(uint32_t(dev::fac_raw<H3D_BF16_SCALED>(p)) << 16);
    }
};

template <int MT> struct S1Slot {
    float a[MT], b[4];
};

template <int DT, int MT, int D, bool ACC64>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MT == 1 ? 3 : 2)))
    k_s1_ring(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ seg_len,
              const int32_t *__restrict__ seg_off, void *const *__restrict__ seg_ptr,
              const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
              const float *__restrict__ scale2, const float *__restrict__ Xs, int NP,
              float *__restrict__ Z, int panel, const int32_t *__restrict__ leaf_off,
              const int32_t *__restrict__ leaf_of, int shc) {
    using F = typename SFac<DT>::T;
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int r16 = lane & 15, q = lane >> 4;
    const int2 it = items[w];
    const int b = it.x, c0 = it.y * 16 * MT;
    const int len = seg_len[b], k = rank[b];
    if (k <= 0 || len <= 0)
        return;
    const int32_t off = seg_off[b];
    const int64_t col0 = blk_col0[b];
    const F *__restrict__ p = static_cast<const F *>(seg_ptr[b]);
    float sc = 1.f;
    if (DT == H3D_BF16_SCALED)
        sc = scale2[2 * b] * scale2[2 * b + 1];
    int cc[MT];
    bool ac[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int c = c0 + 16 * t + r16;
        ac[t] = c < k;
        cc[t] = min(c, k - 1);
    }
    const int S = (len + 3) >> 2;  // K-steps
    for (int nb = 0; nb < NP; nb += 64) {
        const int ntl = min(4, (NP - nb) / 16);
        f4 C[MT][4];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
        constexpr int A64 = ACC64 ? MT : 1;
        double acc64[A64][4][4];
        if constexpr (ACC64) {
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        acc64[t][N][jj] = 0.0;
        }
        auto fill = [&](int s, S1Slot<MT> &sl) {
            const int jc = min(4 * s + q, len - 1);
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                int64_t ea = int64_t(cc[t]) * len + jc;
                if (panel)  // U_b stored as row panels (adjoint above the chunk level)
                    ea = panel_off(leaf_off, leaf_of, shc, off, k, jc, cc[t]);
                sl.a[t] = SFac<DT>::ld(p + ea);
            }
#pragma unroll
            for (int N = 0; N < 4; ++N)
                sl.b[N] = Xs[(int64_t(off) + jc) * NP + nb + 16 * min(N, ntl - 1) + r16];
        };
        S1Slot<MT> R[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
            fill(d, R[d]);
        int ks = 0;
        for (int s0 = 0; s0 < S; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int s = s0 + d;
                if (s >= S)
                    break;
                const bool aj = 4 * s + q < len;
                float av[MT], bv[4];
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    av[t] = (aj && ac[t]) ? R[d].a[t] : 0.f;
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    bv[N] = (aj && N < ntl) ? R[d].b[N] : 0.f;
#pragma unroll
                for (int t = 0; t < MT; ++t)
#pragma unroll
                    for (int N = 0; N < 4; ++N)
                        C[t][N] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], bv[N], C[t][N], 0,
                                                                       0, 0);
                if constexpr (ACC64) {
                    if (++ks == 64) {
                        ks = 0;
#pragma unroll
                        for (int t = 0; t < MT; ++t)
#pragma unroll
                            for (int N = 0; N < 4; ++N) {
#pragma unroll
                                for (int jj = 0; jj < 4; ++jj)
                                    acc64[t][N][jj] += double(C[t][N][jj]);
                                C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
                            }
                    }
                }
                fill(s + D, R[d]);  // past the end: clamped to the last row
            }
        }
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                if (N < ntl)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int c = c0 + 16 * t + 4 * q + jj;
                        if (c < k) {
                            double v = double(C[t][N][jj]);
                            if constexpr (ACC64)
                                v += acc64[t][N][jj];
                            Z[(col0 + c) * NP + nb + 16 * N + r16] = float(v * sc);
                        }
                    }
    }
}

}  // namespace

int s1_ring_tiles(const Plan &P, int l) {
    const int64_t nbl = P.lvl_blk[l + 1] - P.lvl_blk[l];
    const int mean_rank = nbl > 0 ? int(P.lvl_rank_sum[l] / nbl) : 0;
    return std::min(4, std::max(1, (mean_rank + 15) / 16));
}

void launch_s1_ring(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                    const float *Xs, int NP, float *Z, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int mt = s1_ring_tiles(P, l);
    const bool acc = P.max_box[l] > 256;
    const int panel = int(adjoint && l < P.chunk_level);
    const int32_t *len = adjoint ? P.blk_m : P.blk_n;
    const int32_t *off = adjoint ? P.blk_toff : P.blk_soff;
    void *const *ptr = adjoint ? P.blk_uptr : P.blk_vptr;
    const int shc = 3 * (P.L - P.chunk_level);
    // ring depth: eight K-steps for narrow tiles, four for wide ones or FP64 sums
#define H3D_S1R(DT, MT, A)                                                                      \
    k_s1_ring<DT, MT, (MT <= 2 && !A) ? 8 : 4, A><<<int(nitems), 64, 0, s>>>(                  \
        items, nitems, len, off, ptr, P.blk_rank, P.blk_col0, P.blk_scale, Xs, NP, Z, panel,    \
        P.leaf_off, P.leaf_of, shc)
#define H3D_S1R_MT(DT, A)                                                                       \
    switch (mt) {                                                                               \
    case 1: H3D_S1R(DT, 1, A); break;                                                           \
    case 2: H3D_S1R(DT, 2, A); break;                                                           \
    case 3: H3D_S1R(DT, 3, A); break;                                                           \
    default: H3D_S1R(DT, 4, A); break;                                                          \
    }
    if (P.factor_dtype == H3D_F32) {
        if (acc) {
            H3D_S1R_MT(H3D_F32, true)
        } else {
            H3D_S1R_MT(H3D_F32, false)
        }
    } else {
        if (acc) {
            H3D_S1R_MT(H3D_BF16_SCALED, true)
        } else {
            H3D_S1R_MT(H3D_BF16_SCALED, false)
        }
    }
#undef H3D_S1R_MT
#undef H3D_S1R
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
