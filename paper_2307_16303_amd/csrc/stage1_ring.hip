// Many right-hand sides, FP32/BF16 factors: stage 1 of one level, Z_b = V_b^T
// X_s (forward; the adjoint reads U_b and the target rows), with a deep ring
// of fragment loads.
//
// One wave per (block, 16 MT factor columns), four waves per workgroup on
// consecutive items; forward items run in source-box order, so the blocks of
// one source box (the same rows of X) run side by side on one CU.  MT
// 16-column tiles against the four 16-column right-hand-side tiles, 4 MT FP32
// MFMAs per K-step of four source rows, so every X fragment feeds MT MFMAs and
// every factor fragment four.  The assignment of rows to K slots is free as
// long as both operands follow it: K-step i of a super-step S (16 rows) gives
// the lane of K slot q the row 16 S + 4 q + i, so a lane's factor values of
// the four K-steps are four consecutive rows of its column, one 16-byte
// (FP32) or 8-byte (BF16) load instead of four 4-byte loads that each touch 16
// cache lines.  The fragments of the next D2 super-steps are in flight while
// a step's MFMAs run: the loop is a steady part in which every step refills
// its slot and a tail of fewer than D2 steps without refills, so the compiler
// counts the loads in flight exactly and waits for one slot at a time.  Rows
// past the block are masked where the MFMA uses them; their loads stay inside
// the factor chunk (at most three values past a column, which ends at the next
// column, the next block or the chunk's 256 bytes of slack); columns past the
// rank are computed and not written.  Tile N, column n of the MFMA is
// right-hand side 4 n + N of the group of 64, so a lane's four B values and
// four outputs are contiguous (one 16-byte load or store).  Levels whose boxes
// hold at most 256 points sum each column's rows in FP32 (at most 64 K-steps,
// as the other many-RHS kernels flush); longer ones flush the FP32 tiles into
// FP64 sums every 64 K-steps.  Levels split into row parts keep the split
// kernels.
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

// vectors of 4-byte (FP32) and 2-byte (BF16) alignment: global loads at any
// element offset (the HSA targets run with unaligned access enabled)
typedef float f4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u2a2 __attribute__((ext_vector_type(2), aligned(2)));
template <int DT> struct QLoad;
template <> struct QLoad<H3D_F32> {
    static __device__ __forceinline__ f4 ld(const float *p) {
        const f4a4 v = *(const __attribute__((address_space(1))) f4a4 *)p;
        return f4{v[0], v[1], v[2], v[3]};
    }
};
template <> struct QLoad<H3D_BF16_SCALED> {
    static __device__ __forceinline__ f4 ld(const uint16_t *p) {
        const u2a2 w = *(const __attribute__((address_space(1))) u2a2 *)p;
        return f4{__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xffff0000u),
                  __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xffff0000u)};
    }
};

template <int MT> struct QSlot {
    f4 a[MT];  // rows 16 S + 4 q .. + 3 of this lane's column of tile t
    f4 b[4];   // [K-step i]: right-hand sides 4 r16 .. 4 r16 + 3 of row 16 S + 4 q + i
    int kv;    // PANEL: rows of the chunk box from this super-step's first row
};

template <int DT, int MT, int D2, bool ACC64, bool PANEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s1_quad(const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ seg_len,
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
    const int64_t off = seg_off[b];
    const int64_t col0 = blk_col0[b];
    const F *__restrict__ p = static_cast<const F *>(seg_ptr[b]);
    float sc = 1.f;
    if (DT == H3D_BF16_SCALED)
        sc = scale2[2 * b] * scale2[2 * b + 1];
    int cc[MT];  // this lane's factor column of tile t (clamped; outputs past k are not written)
#pragma unroll
    for (int t = 0; t < MT; ++t)
        cc[t] = min(c0 + 16 * t + r16, k - 1);
    // tiles holding columns of the block (the others issue no MFMA; their
    // loads stay, so that every step keeps the same count in flight)
    const int nt = __builtin_amdgcn_readfirstlane(min(MT, (k - c0 + 15) >> 4));
    // super-steps.  PANEL (the adjoint above the chunk level): U_b is stored
    // as one row panel per chunk box of the target box, so the rows are taken
    // chunk box by chunk box, each padded to whole super-steps (the count per
    // box from a table), with a scalar cursor over the chunk boxes one ahead.
    const int S = PANEL ? psteps[leaf_of[off] >> shl] : (len + 15) >> 4;
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
        // chunk cursor (PANEL): rows [pr0, pr0 + plen) of chunk box ch, super-step cs
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
            if (16 * ++cs < plen)
                return;
            if (nch > ch_last) {  // past the last chunk: stay on its last super-step
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
        auto fill = [&](int s, QSlot<MT> &R) {
            // rows j0 .. j0 + 3 of the block (PANEL: of the chunk box's panel)
            const int rows = PANEL ? plen : len;
            const int j0 = (PANEL ? 16 * cs : 16 * s) + 4 * q;
            const int ja = j0 < rows ? j0 : 0;  // a group wholly past the rows: any rows
            const int64_t base = PANEL ? int64_t(pr0 - off) * k : 0;
            const int64_t r0 = PANEL ? pr0 : off;
#pragma unroll
            for (int t = 0; t < MT; ++t)
                R.a[t] = QLoad<DT>::ld(p + base + int64_t(cc[t]) * rows + ja);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                R.b[i] = *reinterpret_cast<const f4 *>(Xs + (r0 + min(j0 + i, rows - 1)) * NP + bcol);
            if constexpr (PANEL)
                R.kv = plen - 16 * cs;
        };
        auto step = [&](int s, const QSlot<MT> &R) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool aj = PANEL ? 4 * q + i < R.kv : 16 * s + 4 * q + i < len;
                float bv[4];
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    bv[N] = aj ? R.b[i][N] : 0.f;
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    if (t < nt)
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            C[t][N] = __builtin_amdgcn_mfma_f32_16x16x4f32(R.a[t][i], bv[N],
                                                                           C[t][N], 0, 0, 0);
            }
        };
        QSlot<MT> R[D2];
#pragma unroll
        for (int d = 0; d < D2; ++d) {
            fill(d, R[d]);
            if constexpr (PANEL)
                padvance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        // steady part: every step refills its slot (past the end: clamped rows,
        // never consumed); then a tail of fewer than D2 steps without refills
        int s0 = 0, ks = 0;
        for (; s0 + D2 <= S; s0 += D2) {
#pragma unroll
            for (int d = 0; d < D2; ++d) {
                step(s0 + d, R[d]);
                fill(s0 + d + D2, R[d]);
                if constexpr (PANEL)
                    padvance();
                // keep each refill right after its step: the scheduler would
                // otherwise sink the loads of all steps below all the MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (ACC64) {
                ks += 4 * D2;
                if (ks + 4 * D2 > 64) {
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
        for (int d = 0; d < D2; ++d)
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

template <int MT> struct S1Slot {
    float a[MT];
    f4 b;
};

// The same product with a run of G consecutive items per wave, for levels of
// many short columns, one K-step (four rows) per slot: the refill cursor runs
// across the items, so the ring never drains between them.  Each item's
// K-steps are padded to a multiple of
// D (padded steps load the item's last rows again and issue no MFMA), so the
// refill cursor enters the next item at slot 0 and the write-out of an item
// runs outside the unrolled ring; the first D steps of an item are written
// out on their own, so that their waits count the stores of the previous
// item's write-out.
template <int DT, int MT, int D, bool ACC64>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s1_ring_g(const int2 *__restrict__ items, int64_t nitems, int G,
                const int32_t *__restrict__ seg_len, const int32_t *__restrict__ seg_off,
                void *const *__restrict__ seg_ptr, const int32_t *__restrict__ rank,
                const int64_t *__restrict__ blk_col0, const float *__restrict__ scale2,
                const float *__restrict__ Xs, int NP, float *__restrict__ Z) {
    using F = typename SFac<DT>::T;
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
        const F *p;
    };
    auto load_item = [&](int64_t i) {
        const uint64_t v = dev::cload(reinterpret_cast<const uint64_t *>(items + i));
        const int2 it{int(uint32_t(v)), int(uint32_t(v >> 32))};  // (block, column group)
        return Item{it.x, it.y * 16 * MT, dev::cload(seg_len + it.x), dev::cload(rank + it.x),
                    int64_t(dev::cload(seg_off + it.x)),
                    static_cast<const F *>(dev::cload(seg_ptr + it.x))};
    };
    auto padded = [](int len) { return (((len + 3) >> 2) + D - 1) / D * D; };
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        // refill cursor: item fi (fc), padded step fs; the next item's metadata ahead
        int64_t fi = i0;
        Item fc = load_item(fi);
        Item fn = fi + 1 < i1 ? load_item(fi + 1) : fc;
        int fS = padded(fc.len), fs = 0;
        int64_t fcol[MT];  // this lane's first element of each tile's column (clamped)
        auto set_cols = [&] {
#pragma unroll
            for (int t = 0; t < MT; ++t)
                fcol[t] = int64_t(min(fc.c0 + 16 * t + r16, fc.k - 1)) * fc.len;
        };
        set_cols();
        auto fadvance = [&] {
            if (++fs < fS)
                return;
            if (fi + 1 >= i1) {  // past the last item: stay on its last step
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
        auto fill = [&](S1Slot<MT> &R) {
            const int jc = min(4 * fs + q, fc.len - 1);
#pragma unroll
            for (int t = 0; t < MT; ++t)
                R.a[t] = SFac<DT>::ld(fc.p + fcol[t] + jc);
            R.b = *reinterpret_cast<const f4 *>(Xs + (fc.off + jc) * NP + bcol);
        };
        S1Slot<MT> R[D];
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
            auto chunk = [&](int s0) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int s = s0 + d;
                    if (s < S) {
                        const bool aj = 4 * s + q < cc.len;
                        float bv[4];
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            bv[N] = aj ? R[d].b[N] : 0.f;
#pragma unroll
                        for (int t = 0; t < MT; ++t)
                            if (t < nt)  // tiles past the block's columns issue no MFMA
#pragma unroll
                                for (int N = 0; N < 4; ++N)
                                    C[t][N] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                        R[d].a[t], bv[N], C[t][N], 0, 0, 0);
                    }
                    fill(R[d]);
                    fadvance();
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            chunk(0);
            int ks = D;
            for (int s0 = D; s0 < Sp; s0 += D) {
                if constexpr (ACC64) {
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
                chunk(s0);
                ks += D;
            }
            float sc = 1.f;
            if (DT == H3D_BF16_SCALED)
                sc = scale2[2 * cc.b] * scale2[2 * cc.b + 1];
            const int64_t col0 = dev::cload(blk_col0 + cc.b);
            if (4 * r16 < nv) {
#pragma unroll
                for (int t = 0; t < MT; ++t)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int c = cc.c0 + 16 * t + 4 * q + jj;
                        if (c < cc.k) {
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
}

// super-steps of the row panels of every box of level l (sum over its chunk
// boxes of ceil(rows / 16)); sh: 3 (chunk level - l), shc: 3 (L - chunk level)
__global__ void k_panel_steps(int64_t nbox, int sh, int shc, const int32_t *__restrict__ leaf_off,
                              int32_t *__restrict__ steps) {
    const int64_t tb = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tb >= nbox)
        return;
    int64_t sum = 0;
    for (int64_t c = tb << sh; c < (tb + 1) << sh; ++c)
        sum += (leaf_off[(c + 1) << shc] - leaf_off[c << shc] + 15) >> 4;
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
    // one item per wave: a ring of two super-steps (eight K-steps); levels of
    // boxes under 64 points: G items per wave, about 16 waves per SIMD, a ring
    // of eight K-steps (six for three or four tiles, within 256 registers)
    const int G = P.mean_box[l] < 64 ? int(std::max<int64_t>(1, nitems / 16384)) : 1;
    const int nwg = int(((nitems + G - 1) / G + 3) / 4);
#define H3D_S1G(DT, MT, A)                                                                      \
    k_s1_ring_g<DT, MT, (MT <= 2 ? 8 : 6), A><<<nwg, 256, 0, s>>>(                              \
        items, nitems, G, len, off, ptr, P.blk_rank, P.blk_col0, P.blk_scale, Xs, NP, Z)
#define H3D_S1Q(DT, MT, A, PN)                                                                  \
    k_s1_quad<DT, MT, 2, A, PN><<<int((nitems + 3) / 4), 256, 0, s>>>(                          \
        items, nitems, len, off, ptr, P.blk_rank, P.blk_col0, P.blk_scale, Xs, NP, Z,           \
        P.leaf_off, P.leaf_of, shc, 3 * (P.L - l), P.bt_pk[l])
#define H3D_S1R_PN(DT, MT, A)                                                                   \
    if (panel)                                                                                  \
        H3D_S1Q(DT, MT, A, true);                                                               \
    else if (G == 1)                                                                            \
        H3D_S1Q(DT, MT, A, false);                                                              \
    else                                                                                        \
        H3D_S1G(DT, MT, A);
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
#undef H3D_S1Q
#undef H3D_S1G
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
