// Many right-hand sides, FP32/BF16 factors: stage 1 of one level, Z_b = V_b^T
// X_s (forward; the adjoint reads U_b and the target rows), with a deep ring
// of fragment loads.
//
// One wave per (block, 16 MT factor columns), four waves per workgroup on
// consecutive items; forward items run in source-box order, so the blocks of
// one source box (the same rows of X) run side by side on one CU.  MT
// 16-column tiles against the
// four 16-column right-hand-side tiles, 4 MT FP32 MFMAs per K-step of four
// source rows, so every X fragment feeds MT MFMAs and every factor fragment
// four.  The fragments of the next D K-steps are in flight while a step's
// MFMAs run: the loop is a steady part in which every step refills its slot
// and a tail of fewer than D steps without refills, so the compiler counts
// the loads in flight exactly and waits for one slot at a time.  Every load is
// issued from a row and column clamped into the block; rows past the block
// are masked where the MFMA uses them, columns past the rank are computed and
// not written.  Tile N, column n of the MFMA is right-hand side 4 n + N of the
// group of 64, so a lane's four B values and four outputs are contiguous (one
// 16-byte load or store).  Levels whose boxes hold at most 256 points sum each
// column's rows in FP32 (at most 64 K-steps, as the other many-RHS kernels
// flush); longer ones flush the FP32 tiles into FP64 sums every 64 K-steps.
// Levels split into row parts keep the split kernels.
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
    float a[MT];
    f4 b;
    int kv;  // PANEL: rows of the chunk box from this step's first row
};

template <int DT, int MT, int D, bool ACC64, bool PANEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s1_ring(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ seg_len,
              const int32_t *__restrict__ seg_off, void *const *__restrict__ seg_ptr,
              const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
              const float *__restrict__ scale2, const float *__restrict__ Xs, int NP,
              float *__restrict__ Z, const int32_t *__restrict__ leaf_off,
              const int32_t *__restrict__ leaf_of, int shc, int shl,
              const int32_t *__restrict__ psteps) {
    using F = typename SFac<DT>::T;
    const int64_t w = dev::xcd_run(blockIdx.x, gridDim.x) * 4 +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nitems)
        return;
    const int lane = threadIdx.x & 63;
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
    int cc[MT];  // this lane's factor column of tile t (clamped; outputs past k are not written)
#pragma unroll
    for (int t = 0; t < MT; ++t)
        cc[t] = min(c0 + 16 * t + r16, k - 1);
    // K-steps.  PANEL (the adjoint above the chunk level): U_b is stored as one
    // row panel per chunk box of the target box, so the rows are taken chunk
    // box by chunk box, each padded to whole K-steps (the count per box from
    // a table), with a scalar cursor over the chunk boxes one ahead.
    const int S = PANEL ? psteps[leaf_of[off] >> shl] : (len + 3) >> 2;
    const int ch_last = PANEL ? (leaf_of[off + len - 1] >> shc) : 0;
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
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
        // chunk cursor (PANEL): rows [pr0, pr0 + plen) of chunk box ch, step cs
        int ch = 0, cs = 0, pr0 = 0, plen = 1, nch = 0, npr0 = 0, nplen = 1;
        auto chunk_rows = [&](int c, int &r0, int &n) {
            r0 = dev::cload(leaf_off + (int64_t(c) << shc));
            n = dev::cload(leaf_off + (int64_t(c + 1) << shc)) - r0;
        };
        auto next_chunk = [&](int c) {  // next chunk box with rows after c (ch_last + 1: none)
            int r0, n;
            for (++c; c <= ch_last; ++c) {
                chunk_rows(c, r0, n);
                if (n > 0)
                    break;
            }
            return c;
        };
        if constexpr (PANEL) {
            ch = leaf_of[off] >> shc;
            chunk_rows(ch, pr0, plen);
            nch = next_chunk(ch);
            if (nch <= ch_last)
                chunk_rows(nch, npr0, nplen);
        }
        auto padvance = [&] {
            if (4 * ++cs < plen)
                return;
            if (nch > ch_last) {  // past the last chunk: stay on its last step
                --cs;
                return;
            }
            ch = nch;
            pr0 = npr0;
            plen = nplen;
            cs = 0;
            nch = next_chunk(ch);
            if (nch <= ch_last)
                chunk_rows(nch, npr0, nplen);
        };
        auto fill = [&](int s, S1Slot<MT> &sl) {
            if constexpr (PANEL) {
                const int lr = min(4 * cs + q, plen - 1);
                const int64_t base = int64_t(pr0 - off) * k + lr;
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    sl.a[t] = SFac<DT>::ld(p + base + int64_t(cc[t]) * plen);
                sl.b = *reinterpret_cast<const f4 *>(Xs + (int64_t(pr0) + lr) * NP + bcol);
                sl.kv = plen - 4 * cs;
            } else {
                const int jc = min(4 * s + q, len - 1);
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    sl.a[t] = SFac<DT>::ld(p + int64_t(cc[t]) * len + jc);
                sl.b = *reinterpret_cast<const f4 *>(Xs + (int64_t(off) + jc) * NP + bcol);
            }
        };
        auto step = [&](int s, const S1Slot<MT> &sl) {
            const bool aj = PANEL ? q < sl.kv : 4 * s + q < len;
            float bv[4];
#pragma unroll
            for (int N = 0; N < 4; ++N)
                bv[N] = aj ? sl.b[N] : 0.f;
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C[t][N] = __builtin_amdgcn_mfma_f32_16x16x4f32(sl.a[t], bv[N], C[t][N], 0, 0, 0);
        };
        S1Slot<MT> R[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            fill(d, R[d]);
            if constexpr (PANEL)
                padvance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        // steady part: every step refills its slot (past the end: clamped rows,
        // never consumed); then a tail of fewer than D steps without refills
        int s0 = 0, ks = 0;
        for (; s0 + D <= S; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                step(s0 + d, R[d]);
                fill(s0 + d + D, R[d]);
                if constexpr (PANEL)
                    padvance();
                // keep each refill right after its step: the scheduler would
                // otherwise sink the loads of all steps below all the MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (ACC64) {
                ks += D;
                if (ks + D > 64) {
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
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (s0 + d < S)
                step(s0 + d, R[d]);
        if (4 * r16 < nv) {
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int c = c0 + 16 * t + 4 * q + jj;
                    if (c < k) {
                        f4 o;
#pragma unroll
                        for (int N = 0; N < 4; ++N) {
                            double v = double(C[t][N][jj]);
                            if constexpr (ACC64)
                                v += acc64[t][N][jj];
                            o[N] = float(v * sc);
                        }
                        *reinterpret_cast<f4 *>(Z + (col0 + c) * NP + nb + 4 * r16) = o;
                    }
                }
        }
    }
}

// K-steps of the row panels of every box of level l (sum over its chunk boxes
// of ceil(rows / 4)); sh: 3 (chunk level - l), shc: 3 (L - chunk level)
__global__ void k_panel_steps(int64_t nbox, int sh, int shc, const int32_t *__restrict__ leaf_off,
                              int32_t *__restrict__ steps) {
    const int64_t tb = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tb >= nbox)
        return;
    int64_t sum = 0;
    for (int64_t c = tb << sh; c < (tb + 1) << sh; ++c)
        sum += (leaf_off[(c + 1) << shc] - leaf_off[c << shc] + 3) >> 2;
    steps[tb] = int32_t(sum);
}

}  // namespace

int32_t *panel_steps(Plan &P, int l, hipStream_t s) {
    const int64_t nbox = pow8(l);
    int32_t *out = P.mem.alloc_n<int32_t>(std::max<int64_t>(nbox, 1));
    k_panel_steps<<<grid_for(nbox, 256), 256, 0, s>>>(nbox, 3 * (P.chunk_level - l),
                                                     3 * (P.L - P.chunk_level), P.leaf_off, out);
    H3D_LAUNCH_CHECK();
    return out;
}

int s1_ring_tiles(const Plan &P, int l) {
    const int64_t nbl = P.lvl_blk[l + 1] - P.lvl_blk[l];
    const int mean_rank = nbl > 0 ? int(P.lvl_rank_sum[l] / nbl) : 0;
    // levels with FP64 sums carry 32 more registers per tile: at most two tiles
    const int cap = P.max_box[l] > 256 ? 2 : 4;
    return std::min(cap, std::max(1, (mean_rank + 15) / 16));
}

void launch_s1_ring(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                    const float *Xs, int NP, float *Z, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int mt = s1_ring_tiles(P, l);
    const bool acc = P.max_box[l] > 256;
    const bool panel = adjoint && l < P.chunk_level;
    const int32_t *len = adjoint ? P.blk_m : P.blk_n;
    const int32_t *off = adjoint ? P.blk_toff : P.blk_soff;
    void *const *ptr = adjoint ? P.blk_uptr : P.blk_vptr;
    const int shc = 3 * (P.L - P.chunk_level);
    // ring of eight K-steps (six for three or four tiles, within 256 registers)
#define H3D_S1R(DT, MT, A, PN)                                                                  \
    k_s1_ring<DT, MT, (MT <= 2 ? 8 : 6), A, PN><<<int((nitems + 3) / 4), 256, 0, s>>>(         \
        items, nitems, len, off, ptr, P.blk_rank, P.blk_col0, P.blk_scale, Xs, NP, Z,           \
        P.leaf_off, P.leaf_of, shc, 3 * (P.L - l), P.bt_pk[l])
#define H3D_S1R_PN(DT, MT, A)                                                                   \
    if (panel)                                                                                  \
        H3D_S1R(DT, MT, A, true);                                                               \
    else                                                                                        \
        H3D_S1R(DT, MT, A, false);
#define H3D_S1R_DT(DT)                                                                          \
    if (acc) {                                                                                  \
        if (mt == 1) {                                                                          \
            H3D_S1R_PN(DT, 1, true)                                                             \
        } else {                                                                                \
            H3D_S1R_PN(DT, 2, true)                                                             \
        }                                                                                       \
    } else {                                                                                    \
        switch (mt) {                                                                           \
        case 1: H3D_S1R_PN(DT, 1, false) break;                                                 \
        case 2: H3D_S1R_PN(DT, 2, false) break;                                                 \
        case 3: H3D_S1R_PN(DT, 3, false) break;                                                 \
        default: H3D_S1R_PN(DT, 4, false) break;                                                \
        }                                                                                       \
    }
    if (P.factor_dtype == H3D_F32) {
        H3D_S1R_DT(H3D_F32)
    } else {
        H3D_S1R_DT(H3D_BF16_SCALED)
    }
#undef H3D_S1R_DT
#undef H3D_S1R_PN
#undef H3D_S1R
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
