// Many right-hand sides, FP32/BF16 factors: stage 2 of one level, Y_t +=
// sum_b U_b Z_b, with a deep ring of fragment loads.
//
// One wave per (target box, 64-row tile): four 16-row tiles M against the
// four 16-column right-hand-side tiles N, 16 FP32 MFMAs per K-step of four
// factor columns, so every fragment loaded feeds four MFMAs.  The K-steps run
// over the columns of all blocks of the box in block order; a cursor walks
// (block, first column) through the blocks' metadata, staged 64 blocks at a
// time in LDS, and the fragments of the next D K-steps are in flight while a
// step's MFMAs run (the ring crosses block boundaries, so it never drains
// inside a box).  Every load is issued from indices clamped into its block
// (past the last block: the last block's first column), and the values are
// masked where the MFMA uses them.  The FP32 tiles are added into the FP64
// rows of Y (read, add, write; each element belongs to one wave) at least
// every 64 K-steps.
#include "product_items.hpp"

namespace h3d {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int DT> struct RFac;
template <> struct RFac<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p) { return dev::fac_raw<H3D_F32>(p); }
};
template <> struct RFac<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ float ld(const T *p) {
        return __uint_as_float(uint32_t(dev::fac_raw<H3D_BF16_SCALED>(p)) << 16);
    }
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Slot {
    float a[4], b[4];
    int kv;  // columns of the step still inside the block (<= 0: past the end)
};

template <int DT, int D>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
    k_s2_ring(const int2 *__restrict__ items, int64_t nitems, int64_t gbase,
              const int32_t *__restrict__ leaf_off, int sh, const int64_t *__restrict__ grp_begin,
              const int64_t *__restrict__ grp_blk, void *const *__restrict__ fptr,
              const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
              const float *__restrict__ Z, int NP, double *__restrict__ Y, int panel,
              const int32_t *__restrict__ leaf_of, int shc) {
    using F = typename RFac<DT>::T;
    __shared__ int32_t s_bk[64];
    __shared__ int64_t s_bc[64];
    __shared__ const F *s_bp[64];
    const int64_t w = blockIdx.x;
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int r16 = lane & 15, q = lane >> 4;
    const int2 it = items[w];
    const int64_t tb = it.x;
    const int32_t bs = leaf_off[tb << sh], bm = leaf_off[(tb + 1) << sh] - bs;
    const int64_t e0 = grp_begin[gbase + tb], e1 = grp_begin[gbase + tb + 1];
    if (e1 <= e0)
        return;
    const int r0 = it.y * 64;
    int iac[4];
    bool ar[4];
    int32_t poff[4], pld[4];  // element (row, c) of U_b at base + poff * k + c * pld
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int i = r0 + 16 * t + r16;
        ar[t] = i < bm;
        iac[t] = min(i, bm - 1);
        int32_t pr0 = bs, ld = bm;
        if (panel) {  // row panels: this row's chunk box
            const int32_t ch = leaf_of[bs + iac[t]] >> shc;
            pr0 = leaf_off[ch << shc];
            ld = leaf_off[(ch + 1) << shc] - pr0;
        }
        poff[t] = pr0 - bs;
        pld[t] = ld;
        iac[t] = bs + iac[t] - pr0;  // row inside the panel
    }
    for (int nb = 0; nb < NP; nb += 64) {
        const int ntl = min(4, (NP - nb) / 16);
        // block cursor over the box's blocks, their metadata 64 at a time in
        // LDS; the current block's pointer, first z index and rank in registers
        int64_t qw = e0;
        int nbk = 0, ib = -1, c = 0;
        bool done = false;
        const F *lbase = nullptr;
        int64_t lcol0 = 0;
        int lk = 1;
        auto stage = [&](int64_t q0) {
            nbk = int(min<int64_t>(64, e1 - q0));
            wave_sync();
            if (lane < nbk) {
                const int64_t bj = grp_blk ? grp_blk[q0 + lane] : q0 + lane;
                s_bk[lane] = rank[bj];
                s_bc[lane] = blk_col0[bj];
                s_bp[lane] = static_cast<const F *>(fptr[bj]);
            }
            wave_sync();
        };
        auto next_block = [&] {  // the next block of nonzero rank, or done
            for (;;) {
                if (++ib >= nbk) {
                    qw += nbk;
                    if (qw >= e1) {
                        done = true;
                        return;
                    }
                    stage(qw);
                    ib = 0;
                }
                const int kk = s_bk[ib];
                if (kk > 0) {
                    lk = kk;
                    lbase = s_bp[ib];
                    lcol0 = s_bc[ib];
                    c = 0;
                    return;
                }
            }
        };
        stage(qw);
        next_block();
        if (done)
            continue;  // every block of the box has rank 0
        // past the end, loads stay on the last block's first column
        auto fill = [&](Slot &S) {
            const int cs = done ? 0 : c;
            S.kv = done ? 0 : lk - c;
            const int cc = min(cs + q, lk - 1);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                S.a[t] = RFac<DT>::ld(lbase + int64_t(poff[t]) * lk + iac[t] + int64_t(cc) * pld[t]);
#pragma unroll
            for (int N = 0; N < 4; ++N)
                S.b[N] = Z[(lcol0 + cc) * NP + nb + 16 * min(N, ntl - 1) + r16];
            if (!done) {
                c += 4;
                if (c >= lk)
                    next_block();
            }
        };
        f4 C[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
        int ks = 0;
        auto flush = [&] {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N) {
                    if (N < ntl)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int r = r0 + 16 * t + 4 * q + jj;
                            if (r < bm) {
                                double *yp = Y + (bs + r) * int64_t(NP) + nb + 16 * N + r16;
                                *yp = *yp + double(C[t][N][jj]);
                            }
                        }
                    C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
                }
            ks = 0;
        };
        Slot R[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
            fill(R[d]);
        bool more = true;
        while (more) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if (R[d].kv <= 0) {
                    more = false;
                    break;
                }
                const bool ak = q < R[d].kv;
                float av[4], bv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    av[t] = (ak && ar[t]) ? R[d].a[t] : 0.f;
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    bv[N] = (ak && N < ntl) ? R[d].b[N] : 0.f;
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int N = 0; N < 4; ++N)
                        C[t][N] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], bv[N], C[t][N], 0, 0,
                                                                       0);
                if (++ks == 64)
                    flush();
                fill(R[d]);
            }
        }
        flush();
    }
}

}  // namespace

void launch_s2_ring(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                    const float *Z, int NP, double *Y, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int panel = int(!adjoint && l < P.chunk_level);
    const int64_t *gblk = adjoint ? P.src_blk : nullptr;
    void *const *fp = adjoint ? P.blk_vptr : P.blk_uptr;
    const int shc = 3 * (P.L - P.chunk_level);
#define H3D_S2R(DT)                                                                             \
    k_s2_ring<DT, 8><<<int(nitems), 64, 0, s>>>(items, nitems, P.box_base[l], P.leaf_off,        \
                                                3 * (P.L - l), P.tgt_begin, gblk, fp, P.blk_rank, \
                                                P.blk_col0, Z, NP, Y, panel, P.leaf_of, shc)
    if (P.factor_dtype == H3D_F32)
        H3D_S2R(H3D_F32);
    else
        H3D_S2R(H3D_BF16_SCALED);
#undef H3D_S2R
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
