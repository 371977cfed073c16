// Many right-hand sides, FP64 factors: stage 1 and stage 2 of one level on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64), with the ring structure of
// the FP32 kernels (stage1_ring.hip, stage2_ring.hip): a steady loop in which
// every K-step refills its slot, then a tail, so each MFMA waits for one slot
// of loads only; a scalar block cursor one block ahead in stage 2; four waves
// per workgroup on consecutive items, workgroups renumbered so that each XCD
// takes a contiguous run.  The sums stay in FP64 throughout.
//
// The FP64 MFMA holds element jj of a lane's accumulator at row 4 jj + q
// (q = lane / 16), column lane % 16; its A and B operands are laid out as the
// FP32 ones (row lane % 16 / K slot q, and K slot q / column lane % 16).
// Tile N, column n is right-hand side 4 n + N of the group of 64, so a lane's
// four z (or x) values of a row and four outputs of a row are contiguous.
//
// Stage 1: one wave per (block, 32 factor columns) (two 16-column tiles).
// Stage 2: two waves per (target box, 64-row tile), 32 rows each.
#include "product_items.hpp"

namespace h3d {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) double GF64;

__device__ __forceinline__ d4 mma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kMT64 = 2;  // 16-column tiles per stage-1 wave

struct S1Slot64 {
    double a[kMT64];
    d4 b;
};

template <int D, bool PANEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s1_ring64(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ seg_len,
                const int32_t *__restrict__ seg_off, void *const *__restrict__ seg_ptr,
                const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
                const double *__restrict__ Xs, int NP, double *__restrict__ Z,
                const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ leaf_of,
                int shc) {
    constexpr int MT = kMT64;
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
    const double *__restrict__ p = static_cast<const double *>(seg_ptr[b]);
    int cc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t)
        cc[t] = min(c0 + 16 * t + r16, k - 1);
    const int nt = __builtin_amdgcn_readfirstlane(min(MT, (k - c0 + 15) >> 4));
    const int S = (len + 3) >> 2;
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        d4 C[MT][4];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                C[t][N] = d4{0.0, 0.0, 0.0, 0.0};
        auto fill = [&](int s, S1Slot64 &sl) {
            const int jc = min(4 * s + q, len - 1);
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                int64_t ea = int64_t(cc[t]) * len + jc;
                if constexpr (PANEL)  // U_b stored as row panels (adjoint above the chunk level)
                    ea = panel_off(leaf_off, leaf_of, shc, off, k, jc, cc[t]);
                sl.a[t] = *(GF64 *)(p + ea);
            }
            sl.b = *reinterpret_cast<const d4 *>(Xs + (int64_t(off) + jc) * NP + bcol);
        };
        auto step = [&](int s, const S1Slot64 &sl) {
            const bool aj = 4 * s + q < len;
#pragma unroll
            for (int t = 0; t < MT; ++t)
                if (t < nt)  // tiles past the block's columns issue no MFMA
#pragma unroll
                    for (int N = 0; N < 4; ++N)
                        C[t][N] = mma64(sl.a[t], aj ? sl.b[N] : 0.0, C[t][N]);
        };
        S1Slot64 R[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            fill(d, R[d]);
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        int s0 = 0;
        for (; s0 + D <= S; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                step(s0 + d, R[d]);
                fill(s0 + d + D, R[d]);
                __builtin_amdgcn_sched_barrier(0);
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
                    const int c = c0 + 16 * t + 4 * jj + q;
                    if (c < k) {
                        d4 o;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            o[N] = C[t][N][jj];
                        *reinterpret_cast<d4 *>(Z + (col0 + c) * NP + nb + 4 * r16) = o;
                    }
                }
        }
    }
}

// Stage 1 with a run of G consecutive items per wave (levels of many short
// columns): the refill cursor runs across the items, each padded to a
// multiple of D steps, as in the FP32 multi-item kernel.
template <int D>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s1_ring64_g(const int2 *__restrict__ items, int64_t nitems, int G,
                  const int32_t *__restrict__ seg_len, const int32_t *__restrict__ seg_off,
                  void *const *__restrict__ seg_ptr, const int32_t *__restrict__ rank,
                  const int64_t *__restrict__ blk_col0, const double *__restrict__ Xs, int NP,
                  double *__restrict__ Z) {
    constexpr int MT = kMT64;
    const int64_t w = dev::xcd_run(blockIdx.x, gridDim.x) * 4 +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i0 = w * G;
    if (i0 >= nitems)
        return;
    const int64_t i1 = min(i0 + int64_t(G), nitems);
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    struct Item {
        int b, c0, len, k;
        int64_t off;
        const double *p;
    };
    auto load_item = [&](int64_t i) {
        const uint64_t v = dev::cload(reinterpret_cast<const uint64_t *>(items + i));
        const int2 it{int(uint32_t(v)), int(uint32_t(v >> 32))};  // (block, column group)
        return Item{it.x, it.y * 16 * MT, dev::cload(seg_len + it.x), dev::cload(rank + it.x),
                    int64_t(dev::cload(seg_off + it.x)),
                    static_cast<const double *>(dev::cload(seg_ptr + it.x))};
    };
    auto padded = [](int len) { return (((len + 3) >> 2) + D - 1) / D * D; };
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        int64_t fi = i0;
        Item fc = load_item(fi);
        Item fn = fi + 1 < i1 ? load_item(fi + 1) : fc;
        int fS = padded(fc.len), fs = 0;
        int64_t fcol[MT];
        auto set_cols = [&] {
#pragma unroll
            for (int t = 0; t < MT; ++t)
                fcol[t] = int64_t(min(fc.c0 + 16 * t + r16, fc.k - 1)) * fc.len;
        };
        set_cols();
        auto fadvance = [&] {
            if (++fs < fS)
                return;
            if (fi + 1 >= i1) {
                fs = fS - 1;
                return;
            }
            ++fi;
            fc = fn;
            fS = padded(fc.len);
            fs = 0;
            set_cols();
            if (fi + 1 < i1)
                fn = load_item(fi + 1);
        };
        auto fill = [&](S1Slot64 &R) {
            const int jc = min(4 * fs + q, fc.len - 1);
#pragma unroll
            for (int t = 0; t < MT; ++t)
                R.a[t] = *(GF64 *)(fc.p + fcol[t] + jc);
            R.b = *reinterpret_cast<const d4 *>(Xs + (fc.off + jc) * NP + bcol);
        };
        S1Slot64 R[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            fill(R[d]);
            fadvance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        Item cn = load_item(i0);  // the consumed item's metadata, one item ahead
        for (int64_t ci = i0; ci < i1; ++ci) {
            const Item cc = cn;
            if (ci + 1 < i1)
                cn = load_item(ci + 1);
            const int S = (cc.len + 3) >> 2, Sp = padded(cc.len);
            const int nt = min(MT, (cc.k - cc.c0 + 15) >> 4);
            d4 C[MT][4];
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C[t][N] = d4{0.0, 0.0, 0.0, 0.0};
            auto chunk = [&](int s0) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int s = s0 + d;
                    if (s < S) {
                        const bool aj = 4 * s + q < cc.len;
#pragma unroll
                        for (int t = 0; t < MT; ++t)
                            if (t < nt)  // tiles past the block's columns issue no MFMA
#pragma unroll
                                for (int N = 0; N < 4; ++N)
                                    C[t][N] = mma64(R[d].a[t], aj ? R[d].b[N] : 0.0, C[t][N]);
                    }
                    fill(R[d]);
                    fadvance();
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            chunk(0);  // on its own: its waits count the previous item's stores
            for (int s0 = D; s0 < Sp; s0 += D)
                chunk(s0);
            const int64_t col0 = dev::cload(blk_col0 + cc.b);
            if (4 * r16 < nv) {
#pragma unroll
                for (int t = 0; t < MT; ++t)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int c = cc.c0 + 16 * t + 4 * jj + q;
                        if (c < cc.k) {
                            d4 o;
#pragma unroll
                            for (int N = 0; N < 4; ++N)
                                o[N] = C[t][N][jj];
                            *reinterpret_cast<d4 *>(Z + (col0 + c) * NP + nb + 4 * r16) = o;
                        }
                    }
            }
        }
    }
}

struct S2Slot64 {
    double a[2];
    d4 b;
};

template <int D>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s2_ring64(const int2 *__restrict__ items, int64_t nitems, int64_t gbase,
                const int32_t *__restrict__ leaf_off, int sh, const int64_t *__restrict__ grp_begin,
                const int64_t *__restrict__ grp_blk, void *const *__restrict__ fptr,
                const int32_t *__restrict__ rank, const int64_t *__restrict__ blk_col0,
                const int32_t *__restrict__ steps, const double *__restrict__ Z, int NP,
                double *__restrict__ Y, int panel, const int32_t *__restrict__ leaf_of, int shc) {
    const int64_t w = dev::xcd_run(blockIdx.x, gridDim.x) * 4 +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= 2 * nitems)
        return;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    const int2 it = items[w >> 1];
    const int64_t tb = it.x;
    const int S = steps[tb];
    if (S <= 0)
        return;
    const int32_t bs = leaf_off[tb << sh], bm = leaf_off[(tb + 1) << sh] - bs;
    const int64_t e0 = grp_begin[gbase + tb], e1 = grp_begin[gbase + tb + 1];
    const int r0 = it.y * 64 + 32 * int(w & 1);
    if (r0 >= bm)
        return;
    int32_t iac[2], poff[2], pld[2];  // element (row, c) of U_b at base + poff k + iac + c pld
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int i = min(r0 + 16 * t + r16, bm - 1);
        int32_t pr0 = bs, ld = bm;
        if (panel) {  // row panels: this row's chunk box
            const int32_t ch = leaf_of[bs + i] >> shc;
            pr0 = leaf_off[ch << shc];
            ld = leaf_off[(ch + 1) << shc] - pr0;
        }
        poff[t] = pr0 - bs;
        pld[t] = ld;
        iac[t] = bs + i - pr0;
    }
    struct Blk {
        int k;
        const double *p;
        int64_t col0;
    };
    auto load = [&](int64_t qq) {
        const int64_t bj = grp_blk ? dev::cload(grp_blk + qq) : qq;
        return Blk{dev::cload(rank + bj), static_cast<const double *>(dev::cload(fptr + bj)),
                   dev::cload(blk_col0 + bj)};
    };
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        // the accumulators start from this wave's rows of Y (rows past the box:
        // the last row, not written back)
        d4 C[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int r = min(r0 + 16 * t + 4 * jj + q, bm - 1);
                const d4 yv = *reinterpret_cast<const d4 *>(Y + (bs + r) * int64_t(NP) + bcol);
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C[t][N][jj] = yv[N];
            }
        int64_t qn = e0;
        Blk cur = load(qn);
        ++qn;
        while (cur.k <= 0 && qn < e1) {
            cur = load(qn);
            ++qn;
        }
        Blk nxt = qn < e1 ? load(qn) : cur;
        int c = 0;
        int32_t roff[2];
        auto set_rows = [&] {
#pragma unroll
            for (int t = 0; t < 2; ++t)
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
        };
        auto fill = [&](S2Slot64 &R) {
            const int cc = min(c + q, cur.k - 1);
#pragma unroll
            for (int t = 0; t < 2; ++t)
                R.a[t] = *(GF64 *)(cur.p + roff[t] + int64_t(cc) * pld[t]);
            R.b = *reinterpret_cast<const d4 *>(Z + (cur.col0 + cc) * NP + bcol);
        };
        S2Slot64 R[D];
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
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C[t][N] = mma64(R[d].a[t], ak ? R[d].b[N] : 0.0, C[t][N]);
        };
        int s0 = 0;
        for (; s0 + D <= S; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                step(d);
                kv[d] = cur.k - c;
                fill(R[d]);
                advance();
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (s0 + d < S)
                step(d);
        if (4 * r16 < nv) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = r0 + 16 * t + 4 * jj + q;
                    if (r < bm) {
                        d4 o;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            o[N] = C[t][N][jj];
                        *reinterpret_cast<d4 *>(Y + (bs + r) * int64_t(NP) + nb + 4 * r16) = o;
                    }
                }
        }
    }
}

}  // namespace

void launch_s1_ring64(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                      const double *Xs, int NP, double *Z, hipStream_t s) {
    if (nitems <= 0)
        return;
    const bool panel = adjoint && l < P.chunk_level;
    const int32_t *len = adjoint ? P.blk_m : P.blk_n;
    const int32_t *off = adjoint ? P.blk_toff : P.blk_soff;
    void *const *ptr = adjoint ? P.blk_uptr : P.blk_vptr;
    const int shc = 3 * (P.L - P.chunk_level);
    if (panel) {
        k_s1_ring64<8, true><<<int((nitems + 3) / 4), 256, 0, s>>>(
            items, nitems, len, off, ptr, P.blk_rank, P.blk_col0, Xs, NP, Z, P.leaf_off,
            P.leaf_of, shc);
    } else if (P.mean_box[l] >= 64) {  // one item per wave (faster for longer columns)
        k_s1_ring64<8, false><<<int((nitems + 3) / 4), 256, 0, s>>>(
            items, nitems, len, off, ptr, P.blk_rank, P.blk_col0, Xs, NP, Z, P.leaf_off,
            P.leaf_of, shc);
    } else {
        // levels of boxes under 64 points: G items per wave, about 16 waves per SIMD
        const int G = int(std::max<int64_t>(1, nitems / 16384));
        k_s1_ring64_g<8><<<int(((nitems + G - 1) / G + 3) / 4), 256, 0, s>>>(
            items, nitems, G, len, off, ptr, P.blk_rank, P.blk_col0, Xs, NP, Z);
    }
    H3D_LAUNCH_CHECK();
}

void launch_s2_ring64(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                      const double *Z, int NP, double *Y, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int panel = int(!adjoint && l < P.chunk_level);
    k_s2_ring64<6><<<int((2 * nitems + 3) / 4), 256, 0, s>>>(
        items, nitems, P.box_base[l], P.leaf_off, 3 * (P.L - l), P.tgt_begin,
        adjoint ? P.src_blk : nullptr, adjoint ? P.blk_vptr : P.blk_uptr, P.blk_rank, P.blk_col0,
        P.bt_s2k[l][adjoint ? 1 : 0], Z, NP, Y, panel, P.leaf_of, 3 * (P.L - P.chunk_level));
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
