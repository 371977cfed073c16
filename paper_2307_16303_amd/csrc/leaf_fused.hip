// Many right-hand sides, finest level, leaves of 17 to 64 rows: both stages
// of every block of a target leaf in one wave, with z never leaving the
// registers.
//
// For a block b of leaf t (source leaf s, n sources, rank k <= 64):
//   stage 1  Z_b = V_b^T X_s     (k x 64): tiles T (16 factor columns) x N
//            (16 right-hand sides), K over the n source rows;
//   stage 2  Y_t += U_b Z_b      (m x 64): tiles M (16 rows) x N, K over the
//            k factor columns.
// On the 16x16x4 FP32 matrix core a lane holds element jj of its accumulator
// at row 4 (lane / 16) + jj, column lane % 16; the B operand of a K-step is
// the element at row lane / 16 of the four K rows.  Taking stage 2's K-steps
// as (T, jj) with the K rows 16 T + 4 q + jj (q = lane / 16), the B operand of
// step (T, jj) is exactly element jj of stage 1's accumulator T: stage 1's
// results feed stage 2 in place, without LDS or memory.  Stage 2's A operand
// is then U_b's column 16 T + 4 q + jj.  Each block's FP32 stage-2 tiles (at
// most 64 columns) are added into FP64 sums of the leaf's rows, which start
// from Y (the near field and the coarser levels) and are written back once.
//
// One wave per leaf; leaves grouped by their 16-row tile count MT, one launch
// per group (a block's rank is at most its leaf's row count, so it has at
// most MT column tiles).  Every load is issued from indices clamped into the block and
// masked where the MFMA uses it.
#include "product_items.hpp"

namespace h3d {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int DT> struct LFac;
template <> struct LFac<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p) { return dev::fac_raw<H3D_F32>(p); }
};
template <> struct LFac<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ float ld(const T *p) {
        return __uint_as_float(uint32_t(dev::fac_raw<H3D_BF16_SCALED>(p)) << 16);
    }
};

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int DT, int MT>
__global__ void __launch_bounds__(64)
    __attribute__((amdgpu_waves_per_eu(MT == 1 ? 4 : (MT <= 3 ? 2 : 1))))
    k_leaf_fused(const int32_t *__restrict__ items, int64_t nitems, int64_t gbase,
                 const int32_t *__restrict__ leaf_off, const int64_t *__restrict__ grp_begin,
                 void *const *__restrict__ uptr, void *const *__restrict__ vptr,
                 const int32_t *__restrict__ rank, const int32_t *__restrict__ soff,
                 const int32_t *__restrict__ slen, const float *__restrict__ scale2,
                 const float *__restrict__ Xs, int NP, double *__restrict__ Y) {
    using F = typename LFac<DT>::T;
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int r16 = lane & 15, q = lane >> 4;
    const int64_t t = items[w];
    const int32_t bs = leaf_off[t], bm = leaf_off[t + 1] - bs;
    const int64_t e0 = grp_begin[gbase + t], e1 = grp_begin[gbase + t + 1];
    int ic[MT];  // this lane's A row of stage-2 tile M, clamped into the leaf
    bool ai[MT];
#pragma unroll
    for (int M = 0; M < MT; ++M) {
        const int i = 16 * M + r16;
        ai[M] = i < bm;
        ic[M] = min(i, bm - 1);
    }
    for (int nb = 0; nb < NP; nb += 64) {
        const int ntl = min(4, (NP - nb) / 16);
        // the leaf's rows of Y in FP64; each block's FP32 tiles are added into
        // them after the block
        double acc64[MT][4][4];
#pragma unroll
        for (int M = 0; M < MT; ++M)
#pragma unroll
            for (int N = 0; N < 4; ++N)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = 16 * M + 4 * q + jj;
                    acc64[M][N][jj] = (N < ntl && r < bm)
                                          ? Y[(bs + r) * int64_t(NP) + nb + 16 * N + r16]
                                          : 0.0;
                }
        for (int64_t b = e0; b < e1; ++b) {
            const int k = rank[b];
            if (k <= 0)
                continue;
            const int n = slen[b];
            const int64_t so = soff[b];
            const F *__restrict__ V = static_cast<const F *>(vptr[b]);
            const F *__restrict__ U = static_cast<const F *>(uptr[b]);
            const int KT = (k + 15) >> 4;
            // ---- stage 1: C1[T][N] = (V^T X)[16 T .., 16 N ..]; k <= m, so
            // the block has at most MT column tiles
            f4 C1[MT][4];
#pragma unroll
            for (int T = 0; T < MT; ++T)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C1[T][N] = f4{0.f, 0.f, 0.f, 0.f};
            int cc[MT];
            bool ac[MT];
#pragma unroll
            for (int T = 0; T < MT; ++T) {
                const int c = 16 * T + r16;
                ac[T] = c < k;
                cc[T] = min(c, k - 1);
            }
            auto frag1 = [&](int s, float (&a)[MT], float (&x)[4]) {
                const int jc = min(4 * s + q, n - 1);
#pragma unroll
                for (int T = 0; T < MT; ++T)
                    a[T] = T < KT ? LFac<DT>::ld(V + int64_t(cc[T]) * n + jc) : 0.f;
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    x[N] = Xs[(so + jc) * NP + nb + 16 * min(N, ntl - 1) + r16];
            };
            const int S1 = (n + 3) >> 2;
            float a0[MT], x0[4], a1[MT], x1[4];
            frag1(0, a0, x0);
            auto step1 = [&](int s, const float (&a)[MT], const float (&x)[4]) {
                const bool aj = 4 * s + q < n;
#pragma unroll
                for (int T = 0; T < MT; ++T)
                    if (T < KT) {
                        const float av = (aj && ac[T]) ? a[T] : 0.f;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            C1[T][N] = mma(av, (aj && N < ntl) ? x[N] : 0.f, C1[T][N]);
                    }
            };
            for (int s = 0; s < S1; s += 2) {
                if (s + 1 < S1)
                    frag1(s + 1, a1, x1);
                step1(s, a0, x0);
                if (s + 1 >= S1)
                    break;
                if (s + 2 < S1)
                    frag1(s + 2, a0, x0);
                step1(s + 1, a1, x1);
            }
            if constexpr (DT == H3D_BF16_SCALED) {
                const float sc = scale2[2 * b] * scale2[2 * b + 1];
#pragma unroll
                for (int T = 0; T < MT; ++T)
#pragma unroll
                    for (int N = 0; N < 4; ++N)
                        C1[T][N] *= sc;
            }
            // ---- stage 2: C2[M][N] = U[16 M .., 16 T + 4 q + jj] C1[T][N][jj]
            f4 C2[MT][4];
#pragma unroll
            for (int M = 0; M < MT; ++M)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C2[M][N] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int T = 0; T < MT; ++T) {
                if (T >= KT)
                    break;
                float u[4][MT];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int c = min(16 * T + 4 * q + jj, k - 1);
#pragma unroll
                    for (int M = 0; M < MT; ++M)
                        u[jj][M] = LFac<DT>::ld(U + int64_t(c) * bm + ic[M]);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const bool kc = 16 * T + 4 * q + jj < k;
#pragma unroll
                    for (int M = 0; M < MT; ++M) {
                        const float av = (kc && ai[M]) ? u[jj][M] : 0.f;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            C2[M][N] = mma(av, C1[T][N][jj], C2[M][N]);
                    }
                }
            }
#pragma unroll
            for (int M = 0; M < MT; ++M)
#pragma unroll
                for (int N = 0; N < 4; ++N)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        acc64[M][N][jj] += double(C2[M][N][jj]);
        }
#pragma unroll
        for (int M = 0; M < MT; ++M)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                if (N < ntl)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int r = 16 * M + 4 * q + jj;
                        if (r < bm)
                            Y[(bs + r) * int64_t(NP) + nb + 16 * N + r16] = acc64[M][N][jj];
                    }
    }
}

}  // namespace

// Leaves of the finest level grouped by 16-row tile count (1..4); false when
// some leaf holds more than 64 rows (the fused form then does not apply).
bool leaf_fused_tables(Plan &P, hipStream_t s) {
    if (P.lf_ready)
        return P.lf_ok;
    P.lf_ready = true;
    P.lf_ok = false;
    const int L = P.L;
    // a block of the finest level has rank <= min(m, n) <= 64 once every leaf
    // holds at most 64 rows
    if (L < 1)
        return false;
    const int64_t nl = pow8(L);
    std::vector<int32_t> cls[4];
    for (int64_t t = 0; t < nl; ++t) {
        const int m = P.h_leaf_off[size_t(t) + 1] - P.h_leaf_off[size_t(t)];
        if (m > 64)
            return false;
        if (m > 0)
            cls[(m - 1) >> 4].push_back(int32_t(t));
    }
    for (int c = 0; c < 4; ++c) {
        P.lf_n[c] = int64_t(cls[c].size());
        P.lf_items[c] = P.mem.alloc_n<int32_t>(std::max<int64_t>(P.lf_n[c], 1));
        if (P.lf_n[c] > 0)
            H3D_HIP(hipMemcpyAsync(P.lf_items[c], cls[c].data(), sizeof(int32_t) * cls[c].size(),
                                   hipMemcpyHostToDevice, s));
    }
    H3D_HIP(hipStreamSynchronize(s));
    P.lf_ok = true;
    return true;
}

void launch_leaf_fused(Plan &P, const float *Xs, int NP, double *Y, hipStream_t s) {
    const int l = P.L;
#define H3D_LF(DT, MT)                                                                          \
    k_leaf_fused<DT, MT><<<int(P.lf_n[MT - 1]), 64, 0, s>>>(                                    \
        P.lf_items[MT - 1], P.lf_n[MT - 1], P.box_base[l], P.leaf_off, P.tgt_begin, P.blk_uptr,  \
        P.blk_vptr, P.blk_rank, P.blk_soff, P.blk_n, P.blk_scale, Xs, NP, Y)
    for (int mt = 1; mt <= 4; ++mt) {
        if (P.lf_n[mt - 1] == 0)
            continue;
        if (P.factor_dtype == H3D_F32) {
            switch (mt) {
            case 1: H3D_LF(H3D_F32, 1); break;
            case 2: H3D_LF(H3D_F32, 2); break;
            case 3: H3D_LF(H3D_F32, 3); break;
            default: H3D_LF(H3D_F32, 4); break;
            }
        } else {
            switch (mt) {
            case 1: H3D_LF(H3D_BF16_SCALED, 1); break;
            case 2: H3D_LF(H3D_BF16_SCALED, 2); break;
            case 3: H3D_LF(H3D_BF16_SCALED, 3); break;
            default: H3D_LF(H3D_BF16_SCALED, 4); break;
            }
        }
        H3D_LAUNCH_CHECK();
    }
#undef H3D_LF
}

}  // namespace h3d
