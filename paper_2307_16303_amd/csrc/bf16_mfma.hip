// Many right-hand sides, BF16 factors, forward product: stages 1 and 2 of the
// far field on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16), instead of
// widening the factors to FP32 tiles.
//
// The factors are BF16 already (with a per-block scale); the other operand, x
// in stage 1 and z in stage 2, is carried as two BF16 parts, hi = bf16(v) and
// lo = bf16(v - hi) (packed hi | lo << 16 in one 32-bit word), and every
// product is formed as A hi + A lo on the FP32 accumulator.  hi + lo holds v
// to about 2^-17 relative, so the result is that of the BF16 factors with an
// exact right-hand side up to terms far below the factors' own rounding
// (2^-9).  The accumulators stay in FP32 over a whole block column (stage 1)
// or a whole box (stage 2): at most 2^15 terms, whose FP32 summation error is
// also far below the factors' rounding; y receives each tile once, in FP64.
//
// Fragment layout of the 16x16x16 BF16 MFMA (lane l = 16 q + r16): A holds
// row r16, K slots 4 q .. 4 q + 3; B holds K slots 4 q .. 4 q + 3 of column
// r16; the accumulator holds rows 4 q + jj, column r16.  Tile N, column n is
// right-hand side 4 n + N of a group of 64 (as in the FP32 ring kernels), so
// a lane's four x or z words of a row are one 16-byte load.
//
// Stage 1: one wave per run of G consecutive (block, 16 MT factor columns)
// items, the refill cursor crossing the items (each padded to whole rings);
// a K-step is 16 source rows.  A lane's four K slots are four consecutive rows of a V_b column: one
// 8-byte piece at any 2-byte alignment, read as the three aligned words that
// hold it (the factor chunks end with 256 bytes of slack).
// Stage 2: two waves per (target box, 64-row tile), 32 rows each; a K-step is
// 16 factor columns of one block.  A lane's four K slots are four columns of
// its row of U_b: four 2-byte loads per row tile.
// Both run a ring of D K-steps (a steady part where each step refills its slot,
// then a tail), four waves per workgroup on consecutive items.
#include "product_items.hpp"

namespace h3d {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) uint32_t GU32;
typedef const __attribute__((address_space(1))) uint16_t GU16;

// round to nearest even (finite values)
__device__ __forceinline__ uint32_t bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t split_hl(float f) {
    const uint32_t h = bf16_bits(f);
    return h | (bf16_bits(f - __uint_as_float(h << 16)) << 16);
}

// four BF16 values at p (2-byte aligned) from the three aligned words holding them
__device__ __forceinline__ void ld4_raw(const uint16_t *p, uint32_t (&w)[3], bool &odd) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    GU32 *a4 = (GU32 *)(a & ~uintptr_t(3));
    __builtin_memcpy(w, (const uint32_t *)a4, 12);
    odd = (a & 2) != 0;
}
__device__ __forceinline__ s4 fix4(const uint32_t (&w)[3], bool odd, uint32_t keep_lo,
                                   uint32_t keep_hi) {
    uint32_t d0 = odd ? __builtin_amdgcn_alignbit(w[1], w[0], 16) : w[0];
    uint32_t d1 = odd ? __builtin_amdgcn_alignbit(w[2], w[1], 16) : w[1];
    d0 &= keep_lo;
    d1 &= keep_hi;
    s4 r;
    const uint64_t v = uint64_t(d0) | (uint64_t(d1) << 32);
    __builtin_memcpy(&r, &v, 8);
    return r;
}
// B operands of tile N from the four K-slot rows' words (hi | lo << 16)
// (v_perm_b32 selects bytes of {first, second}: 0-3 from the second, 4-7 from the first)
__device__ __forceinline__ s4 pack_hi(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3) {
    const uint64_t v = uint64_t(__builtin_amdgcn_perm(x1, x0, 0x05040100u)) |
                       (uint64_t(__builtin_amdgcn_perm(x3, x2, 0x05040100u)) << 32);
    s4 r;
    __builtin_memcpy(&r, &v, 8);
    return r;
}
__device__ __forceinline__ s4 pack_lo(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3) {
    const uint64_t v = uint64_t(__builtin_amdgcn_perm(x1, x0, 0x07060302u)) |
                       (uint64_t(__builtin_amdgcn_perm(x3, x2, 0x07060302u)) << 32);
    s4 r;
    __builtin_memcpy(&r, &v, 8);
    return r;
}
__device__ __forceinline__ f4 mma(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// mask keeping the K slots i with valid (bit i) set, for the two words of a s4
__device__ __forceinline__ void slot_masks(int nvalid, uint32_t &lo, uint32_t &hi) {
    lo = (nvalid >= 2 ? 0xffffffffu : (nvalid == 1 ? 0xffffu : 0u));
    hi = (nvalid >= 4 ? 0xffffffffu : (nvalid == 3 ? 0xffffu : 0u));
}

template <int MT> struct S1Slot {
    uint32_t a[MT][3];
    bool odd[MT];
    u4 x[4];
};

template <int MT, int D>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s1_bf16(const int2 *__restrict__ items, int64_t nitems, int G,
              const int32_t *__restrict__ seg_len, const int32_t *__restrict__ seg_off,
              void *const *__restrict__ seg_ptr, const int32_t *__restrict__ rank,
              const int64_t *__restrict__ blk_col0, const float *__restrict__ scale2,
              const uint32_t *__restrict__ Xh, int NP, uint32_t *__restrict__ Zh) {
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
        const uint16_t *p;
    };
    auto load_item = [&](int64_t i) {
        const uint64_t v = dev::cload(reinterpret_cast<const uint64_t *>(items + i));
        const int b = int(uint32_t(v)), grp = int(uint32_t(v >> 32));  // (block, column group)
        return Item{b, grp * 16 * MT, dev::cload(seg_len + b), dev::cload(rank + b),
                    int64_t(dev::cload(seg_off + b)),
                    static_cast<const uint16_t *>(dev::cload(seg_ptr + b))};
    };
    auto padded = [](int len) { return (((len + 15) >> 4) + D - 1) / D * D; };
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        // refill cursor (item fi, padded K-step fs of 16 rows), the next item ahead
        int64_t fi = i0;
        Item fc = load_item(fi);
        Item fn = fi + 1 < i1 ? load_item(fi + 1) : fc;
        int fS = padded(fc.len), fs = 0;
        int64_t ce[MT];  // first element of this lane's column of tile T (clamped into the block)
        auto set_cols = [&] {
#pragma unroll
            for (int T = 0; T < MT; ++T)
                ce[T] = int64_t(min(fc.c0 + 16 * T + r16, fc.k - 1)) * fc.len;
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
            const int j0 = min(16 * fs + 4 * q, fc.len - 1);
#pragma unroll
            for (int T = 0; T < MT; ++T)
                ld4_raw(fc.p + ce[T] + j0, R.a[T], R.odd[T]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                R.x[i] = *(const u4 *)((GU32 *)(Xh + (fc.off + min(16 * fs + 4 * q + i, fc.len - 1)) *
                                                         NP +
                                                 bcol));
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
            const int S = (cc.len + 15) >> 4, Sp = padded(cc.len);
            const int nt = min(MT, (cc.k - cc.c0 + 15) >> 4);
            f4 C[MT][4];
#pragma unroll
            for (int T = 0; T < MT; ++T)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C[T][N] = f4{0.f, 0.f, 0.f, 0.f};
            auto step = [&](int s, const S1Slot<MT> &R) {
                uint32_t mlo, mhi;
                slot_masks(cc.len - (16 * s + 4 * q), mlo, mhi);
                s4 bh[4], bl[4];
#pragma unroll
                for (int N = 0; N < 4; ++N) {
                    bh[N] = pack_hi(R.x[0][N], R.x[1][N], R.x[2][N], R.x[3][N]);
                    bl[N] = pack_lo(R.x[0][N], R.x[1][N], R.x[2][N], R.x[3][N]);
                }
#pragma unroll
                for (int T = 0; T < MT; ++T) {
                    if (T >= nt)  // tiles past the block's columns issue no MFMA
                        break;
                    const s4 a = fix4(R.a[T], R.odd[T], mlo, mhi);
#pragma unroll
                    for (int N = 0; N < 4; ++N) {
                        C[T][N] = mma(a, bh[N], C[T][N]);
                        C[T][N] = mma(a, bl[N], C[T][N]);
                    }
                }
            };
            auto chunk = [&](int s0) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (s0 + d < S)
                        step(s0 + d, R[d]);
                    fill(R[d]);
                    fadvance();
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            chunk(0);  // on its own: its waits count the previous item's stores
            for (int s0 = D; s0 < Sp; s0 += D)
                chunk(s0);
            const float sc = scale2[2 * cc.b] * scale2[2 * cc.b + 1];
            const int64_t col0 = dev::cload(blk_col0 + cc.b);
            if (4 * r16 < nv) {
#pragma unroll
                for (int T = 0; T < MT; ++T)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int c = cc.c0 + 16 * T + 4 * q + jj;
                        if (c < cc.k) {
                            u4 o;
#pragma unroll
                            for (int N = 0; N < 4; ++N)
                                o[N] = split_hl(C[T][N][jj] * sc);
                            *reinterpret_cast<u4 *>(Zh + (col0 + c) * NP + nb + 4 * r16) = o;
                        }
                    }
            }
        }
    }
}

struct S2Slot {
    uint16_t a[2][4];  // [tile][K slot]
    u4 z[4];           // [K slot]: the words of right-hand sides 4 r16 .. 4 r16 + 3
    int kv;            // columns of the block from this step's first column
};

template <int D>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_s2_bf16(const int2 *__restrict__ items, int64_t nitems, int64_t gbase,
              const int32_t *__restrict__ leaf_off, int sh, const int64_t *__restrict__ grp_begin,
              void *const *__restrict__ fptr, const int32_t *__restrict__ rank,
              const int64_t *__restrict__ blk_col0, const int32_t *__restrict__ steps,
              const uint32_t *__restrict__ Zh, int NP, double *__restrict__ Y, int panel,
              const int32_t *__restrict__ leaf_of, int shc) {
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
        const uint16_t *p;
        int64_t col0;
    };
    auto load = [&](int64_t qq) {
        return Blk{dev::cload(rank + qq), static_cast<const uint16_t *>(dev::cload(fptr + qq)),
                   dev::cload(blk_col0 + qq)};
    };
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
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
            c += 16;
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
        auto fill = [&](S2Slot &R) {
            R.kv = cur.k - c;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int cc = min(c + 4 * q + i, cur.k - 1);
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    R.a[t][i] = *(GU16 *)(cur.p + roff[t] + int64_t(cc) * pld[t]);
                R.z[i] = *(const u4 *)((GU32 *)(Zh + (cur.col0 + cc) * NP + bcol));
            }
        };
        f4 C[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                C[t][N] = f4{0.f, 0.f, 0.f, 0.f};
        auto step = [&](const S2Slot &R) {
            uint32_t mlo, mhi;
            slot_masks(R.kv - 4 * q, mlo, mhi);
            s4 bh[4], bl[4];
#pragma unroll
            for (int N = 0; N < 4; ++N) {
                bh[N] = pack_hi(R.z[0][N], R.z[1][N], R.z[2][N], R.z[3][N]);
                bl[N] = pack_lo(R.z[0][N], R.z[1][N], R.z[2][N], R.z[3][N]);
            }
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                // low halves of two words: bytes 0-1 of the first, 0-1 of the second
                const uint32_t w0 = __builtin_amdgcn_perm(R.a[t][1], R.a[t][0], 0x05040100u);
                const uint32_t w1 = __builtin_amdgcn_perm(R.a[t][3], R.a[t][2], 0x05040100u);
                const uint64_t v = uint64_t(w0 & mlo) | (uint64_t(w1 & mhi) << 32);
                s4 a;
                __builtin_memcpy(&a, &v, 8);
#pragma unroll
                for (int N = 0; N < 4; ++N) {
                    C[t][N] = mma(a, bh[N], C[t][N]);
                    C[t][N] = mma(a, bl[N], C[t][N]);
                }
            }
        };
        S2Slot R[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            fill(R[d]);
            advance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        int s0 = 0;
        for (; s0 + D <= S; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                step(R[d]);
                fill(R[d]);
                advance();
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (s0 + d < S)
                step(R[d]);
        if (4 * r16 < nv) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = r0 + 16 * t + 4 * q + jj;
                    if (r < bm) {
                        double *yp = Y + (bs + r) * int64_t(NP) + nb + 4 * r16;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            yp[N] += double(C[t][N][jj]);
                    }
                }
        }
    }
}

// K-steps of 16 columns of every box of a level (sum over its blocks of ceil(k_b / 16))
__global__ void k_s2_steps16(int64_t nbox, int64_t gbase, const int64_t *__restrict__ grp_begin,
                             const int32_t *__restrict__ rank, int32_t *__restrict__ steps) {
    const int64_t tb = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tb >= nbox)
        return;
    int64_t sum = 0;
    for (int64_t e = grp_begin[gbase + tb]; e < grp_begin[gbase + tb + 1]; ++e) {
        const int k = rank[e];
        sum += k > 0 ? (k + 15) / 16 : 0;
    }
    steps[tb] = int32_t(sum);
}

// hi | lo << 16 of every FP32 value of x
__global__ void k_split_x(int64_t count, const float *__restrict__ Xs, uint32_t *__restrict__ Xh) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count)
        Xh[i] = split_hl(Xs[i]);
}

}  // namespace

int32_t *s2_bf16_steps(Plan &P, int l, hipStream_t s) {
    const int64_t nbox = pow8(l);
    int32_t *out = P.mem.alloc_n<int32_t>(std::max<int64_t>(nbox, 1));
    k_s2_steps16<<<grid_for(nbox, 256), 256, 0, s>>>(nbox, P.box_base[l], P.tgt_begin, P.blk_rank,
                                                    out);
    H3D_LAUNCH_CHECK();
    return out;
}

void launch_split_x(const float *Xs, int64_t count, uint32_t *Xh, hipStream_t s) {
    if (count <= 0)
        return;
    k_split_x<<<grid_for(count, 256), 256, 0, s>>>(count, Xs, Xh);
    H3D_LAUNCH_CHECK();
}

void launch_s1_bf16(Plan &P, int l, const int2 *items, int64_t nitems, const uint32_t *Xh, int NP,
                    uint32_t *Zh, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int mt = s1_ring_tiles(P, l);
    // levels of boxes under 256 points (under 16 K-steps of 16 rows): G items
    // per wave, about 16 waves per SIMD; one item per wave otherwise
    const int G = P.mean_box[l] < 256 ? int(std::max<int64_t>(1, nitems / 16384)) : 1;
    const int nwg = int(((nitems + G - 1) / G + 3) / 4);
#define H3D_S1B(MT)                                                                             \
    k_s1_bf16<MT, (MT <= 2 ? 4 : (MT == 3 ? 3 : 2))><<<nwg, 256, 0, s>>>(items, nitems, G, P.blk_n, P.blk_soff,  \
                                                         P.blk_vptr, P.blk_rank, P.blk_col0,    \
                                                         P.blk_scale, Xh, NP, Zh)
    switch (mt) {
    case 1: H3D_S1B(1); break;
    case 2: H3D_S1B(2); break;
    case 3: H3D_S1B(3); break;
    default: H3D_S1B(4); break;
    }
#undef H3D_S1B
    H3D_LAUNCH_CHECK();
}

void launch_s2_bf16(Plan &P, int l, const int2 *items, int64_t nitems, const uint32_t *Zh, int NP,
                    double *Y, hipStream_t s) {
    if (nitems <= 0)
        return;
    const int panel = int(l < P.chunk_level);
    const int shc = 3 * (P.L - P.chunk_level);
    k_s2_bf16<4><<<int((2 * nitems + 3) / 4), 256, 0, s>>>(
        items, nitems, P.box_base[l], P.leaf_off, 3 * (P.L - l), P.tgt_begin, P.blk_uptr,
        P.blk_rank, P.blk_col0, P.bt_s2k16[l], Zh, NP, Y, panel, P.leaf_of, shc);
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
