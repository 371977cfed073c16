// Many right-hand sides, FP32/BF16 factors: stage 2 of one level, Y_t +=
// sum_b U_b Z_b, with a deep ring of fragment loads.
//
// One wave per (target box, 64-row tile): four 16-row tiles M against four
// 16-column right-hand-side tiles N, 16 FP32 MFMAs per K-step of four factor
// columns, so every fragment loaded feeds four MFMAs.  Where the factor's
// columns are contiguous over the box's rows (all but the row panels), tile
// t's MFMA row r is row 4 r + t of the 64, so that a lane's four A values of a
// K-step are four consecutive rows of its column, read with one load.  The K-steps run over the
// columns of all blocks of the box in block order; their count S is known from
// a table (sum over the box's blocks of ceil(k_b / 4)), so the loop is a
// steady part in which every step refills its ring slot and a tail without
// refills: the compiler then counts the loads in flight exactly and waits for
// one slot at a time.  The block cursor reads the blocks' rank, factor pointer
// and first z index with scalar loads, one block ahead.  Past the last block
// the loads stay on that block's first columns (never consumed).
//
// Tile N, column n of the MFMA is right-hand side 4 n + N of the group of 64,
// so a lane's four B values (and its four outputs of a row) are contiguous:
// one 16-byte load of z per K-step.  The wave's rows of Y are held in FP64
// registers (read once before the K-steps, written once after them); the FP32
// tiles are added into them at least every 64 K-steps.  Four waves of a
// workgroup take four consecutive items, mostly the row tiles of one box, so
// the box's z fragments are fetched once into the CU's caches for all four.
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

// QUAD: tile t, row r of the MFMA is row r0 + 4 r + t of the tile of 64,
// so a lane's four A values of a K-step are four consecutive rows of one
// factor column (one 16-byte FP32 or 8-byte BF16 load); otherwise row
// r0 + 16 t + r (row panels: a tile may cross chunk boxes).
typedef float f4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u2a2 __attribute__((ext_vector_type(2), aligned(2)));
template <int DT> struct RQuad;
template <> struct RQuad<H3D_F32> {
    static __device__ __forceinline__ f4 ld(const float *p) {
        const f4a4 v = *(const __attribute__((address_space(1))) f4a4 *)p;
        return f4{v[0], v[1], v[2], v[3]};
    }
};
template <> struct RQuad<H3D_BF16_SCALED> {
    static __device__ __forceinline__ f4 ld(const uint16_t *p) {
        const u2a2 w = *(const __attribute__((address_space(1))) u2a2 *)p;
        return f4{__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xffff0000u),
                  __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xffff0000u)};
    }
};

struct Slot {
    f4 a;  // [t]: this lane's A value of tile t
    f4 b;
};

// the Y row of tile t, accumulator element jj of lane quarter q
template <bool QUAD> __device__ __forceinline__ int s2_row(int r0, int t, int q, int jj) {
    return QUAD ? r0 + 16 * q + 4 * jj + t : r0 + 16 * t + 4 * q + jj;
}

template <int DT, int D, bool QUAD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
    k_s2_ring(const int2 *__restrict__ items, int64_t nitems, int64_t gbase,
              const int32_t *__restrict__ leaf_off, int sh, const int64_t *__restrict__ grp_begin,
              const int64_t *__restrict__ grp_blk, void *const *__restrict__ fptr,
              const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
              const int32_t *__restrict__ steps, const float *__restrict__ Z, int NP,
              double *__restrict__ Y, int panel, const int32_t *__restrict__ leaf_of, int shc) {
    using F = typename RFac<DT>::T;
    const int64_t w = dev::xcd_run(blockIdx.x, gridDim.x) * 4 +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nitems)
        return;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    const int2 it = items[w];
    const int64_t tb = it.x;
    const int S = steps[tb];
    if (S <= 0)
        return;
    const int32_t bs = leaf_off[tb << sh], bm = leaf_off[(tb + 1) << sh] - bs;
    const int64_t e0 = grp_begin[gbase + tb], e1 = grp_begin[gbase + tb + 1];
    const int r0 = it.y * 64;
    int32_t iac[4], poff[4], pld[4];  // element (row, c) of U_b at base + poff k + iac + c pld
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        // QUAD: the first of the lane's four rows (a group starting past the
        // box reads any rows of the column: it is never written)
        const int i = min(QUAD ? r0 + 4 * r16 : r0 + 16 * t + r16, bm - 1);
        int32_t pr0 = bs, ld = bm;
        if (panel) {  // row panels: this row's chunk box
            const int32_t ch = leaf_of[bs + i] >> shc;
            pr0 = leaf_off[ch << shc];
            ld = leaf_off[(ch + 1) << shc] - pr0;
        }
        poff[t] = pr0 - bs;
        pld[t] = ld;
        iac[t] = bs + i - pr0;  // row inside the panel
    }
    struct Blk {
        int k;
        const F *p;
        int64_t col0;
    };
    // the block tables are read-only here: constant-space loads stay scalar
    auto load = [&](int64_t qq) {
        const int64_t bj = grp_blk ? dev::cload(grp_blk + qq) : qq;
        return Blk{dev::cload(rank + bj), static_cast<const F *>(dev::cload(fptr + bj)), dev::cload(blk_col0 + bj)};
    };
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        // this wave's rows of Y (rows past the box: the last row, not written)
        double acc64[4][4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int r = min(s2_row<QUAD>(r0, t, q, jj), bm - 1);
                const double *yp = Y + (bs + r) * int64_t(NP) + bcol;
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    acc64[t][jj][N] = yp[N];
            }
        // cursor: current block and column; the next block's metadata in flight
        int64_t qn = e0;
        Blk cur = load(qn);
        ++qn;
        while (cur.k <= 0 && qn < e1) {
            cur = load(qn);
            ++qn;
        }
        Blk nxt = qn < e1 ? load(qn) : cur;
        int c = 0;
        int32_t roff[4];
        auto set_rows = [&] {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                roff[t] = poff[t] * cur.k + iac[t];
        };
        set_rows();
        auto advance = [&] {
            c += 4;
            if (c < cur.k)
                return;
            c = 0;
            while (qn < e1) {
                const Blk b = nxt;
                ++qn;
                if (qn < e1)
                    nxt = load(qn);
                if (b.k > 0) {
                    cur = b;
                    set_rows();
                    return;
                }
            }
            // past the last block: the cursor stays on it
        };
        auto fill = [&](Slot &R) {
            const int cc = min(c + q, cur.k - 1);
            if constexpr (QUAD) {
                // (at most three values past the column: the next column, the
                // next block or the chunk's 256 bytes of slack)
                R.a = RQuad<DT>::ld(cur.p + roff[0] + int64_t(cc) * pld[0]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    R.a[t] = RFac<DT>::ld(cur.p + roff[t] + int64_t(cc) * pld[t]);
            }
            R.b = *reinterpret_cast<const f4 *>(Z + (cur.col0 + cc) * NP + bcol);
        };
        f4 C[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
        auto flush = [&] {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N) {
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
                        acc64[t][jj][N] += double(C[t][N][jj]);
                    C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
                }
        };
        // columns of the step still inside its block (a partial last step of
        // a block has kv < 4)
        Slot R[D];
        int kv[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            kv[d] = cur.k - c;
            fill(R[d]);
            advance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        auto step = [&](int d) {
            const bool ak = q < kv[d];
            float bv[4];
#pragma unroll
            for (int N = 0; N < 4; ++N)
                bv[N] = ak ? R[d].b[N] : 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C[t][N] = __builtin_amdgcn_mfma_f32_16x16x4f32(R[d].a[t], bv[N], C[t][N], 0, 0,
                                                                   0);
        };
        int s0 = 0, ks = 0;
        for (; s0 + D <= S; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                step(d);
                kv[d] = cur.k - c;
                fill(R[d]);
                advance();
                __builtin_amdgcn_sched_barrier(0);
            }
            ks += D;
            if (ks + D > 64) {
                flush();
                ks = 0;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (s0 + d < S)
                step(d);
        flush();
        if (4 * r16 < nv) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = s2_row<QUAD>(r0, t, q, jj);
                    if (r < bm) {
                        double *yp = Y + (bs + r) * int64_t(NP) + nb + 4 * r16;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            yp[N] = acc64[t][jj][N];
                    }
                }
        }
    }
}

// K-steps of every box of a level: sum over its blocks of ceil(k_b / 4)
__global__ void k_s2_steps(int64_t nbox, int64_t gbase, const int64_t *__restrict__ grp_begin,
                           const int64_t *__restrict__ grp_blk, const int32_t *__restrict__ rank,
                           int32_t *__restrict__ steps) {
    const int64_t tb = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tb >= nbox)
        return;
    int64_t sum = 0;
    for (int64_t e = grp_begin[gbase + tb]; e < grp_begin[gbase + tb + 1]; ++e) {
        const int k = rank[grp_blk ? grp_blk[e] : e];
        sum += k > 0 ? (k + 3) / 4 : 0;
    }
    steps[tb] = int32_t(sum);
}

}  // namespace

int32_t *s2_ring_steps(Plan &P, int l, bool adjoint, hipStream_t s) {
    const int64_t nbox = pow8(l);
    int32_t *out = P.mem.alloc_n<int32_t>(std::max<int64_t>(nbox, 1));
    k_s2_steps<<<grid_for(nbox, 256), 256, 0, s>>>(nbox, P.box_base[l], P.tgt_begin,
                                                  adjoint ? P.src_blk : nullptr, P.blk_rank, out);
    H3D_LAUNCH_CHECK();
    return out;
}

void launch_s2_ring(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                    const float *Z, int NP, double *Y, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int panel = int(!adjoint && l < P.chunk_level);
    const int64_t *gblk = adjoint ? P.src_blk : nullptr;
    void *const *fp = adjoint ? P.blk_vptr : P.blk_uptr;
    const int32_t *steps = P.bt_s2k[l][adjoint ? 1 : 0];
    const int shc = 3 * (P.L - P.chunk_level);
#define H3D_S2R(DT, Q)                                                                          \
    k_s2_ring<DT, 8, Q><<<int((nitems + 3) / 4), 256, 0, s>>>(                                  \
        items, nitems, P.box_base[l], P.leaf_off, 3 * (P.L - l), P.tgt_begin, gblk, fp,          \
        P.blk_rank, P.blk_col0, steps, Z, NP, Y, panel, P.leaf_of, shc)
    if (P.factor_dtype == H3D_F32) {
        if (panel)
            H3D_S2R(H3D_F32, false);
        else
            H3D_S2R(H3D_F32, true);
    } else {
        if (panel)
            H3D_S2R(H3D_BF16_SCALED, false);
        else
            H3D_S2R(H3D_BF16_SCALED, true);
    }
#undef H3D_S2R
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
