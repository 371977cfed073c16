// Many right-hand sides, finest level, leaves of at most 64 rows: both stages
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
// the element at row lane / 16 of the four K rows.  Row rho of stage 1's tile
// T is factor column 16 T + 4 (rho % 4) + rho / 4, so element jj of lane q's
// accumulator T is column 16 T + 4 jj + q (q = lane / 16).  Taking stage 2's
// K-steps as (T, jj), with the K rows 16 T + 4 jj .. + 3, the B operand of
// step (T, jj) is exactly element jj of stage 1's accumulator T: stage 1's
// results feed stage 2 in place, without LDS or memory, and a block of rank
// k takes only the K-steps with 16 T + 4 jj < k.  Stage 2's A operand is then
// U_b's column 16 T + 4 jj + q.  Each block's FP32 stage-2 tiles (at
// most 64 columns) are added into FP64 sums of the leaf's rows, which start
// from Y (the near field and the coarser levels) and are written back once.
//
// Loads run ahead of the MFMAs through a ring of D stage-1 super-steps (four
// K-steps, 16 source rows; a lane's four factor values of a super-step are
// consecutive rows of its column, read at once) that crosses blocks: each
// block's super-steps are padded to a multiple of D (padded steps load again
// the block's last rows and issue no MFMA), so the
// refill cursor, exactly D steps ahead, enters the next block at slot 0 and
// stage 2 runs once per block outside the unrolled ring.  The U_b columns of
// the first UP column tiles are loaded when the block's stage 1 begins, the
// others just before use.  The block metadata is read with scalar loads, one
// block ahead.  Tile N, column n of the MFMA is right-hand side 4 n + N of the
// group of 64, so a lane's four X values and four outputs of a row are
// contiguous.
//
// The adjoint is the same product with U and V exchanged: the blocks of a
// source leaf (through the source-grouped block table), stage 1 over the
// target rows with U_b, stage 2 into the source leaf's rows with V_b.
//
// One wave per leaf; leaves grouped by their 16-row tile count MT, one launch
// per group (a block's rank is at most its leaf's row count, so it has at
// most MT column tiles).  Every load is issued from indices clamped into the
// block and masked where the MFMA uses it.
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

// four consecutive factor values of a column (any element alignment; the
// HSA targets run with unaligned access enabled)
typedef float f4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u2a2 __attribute__((ext_vector_type(2), aligned(2)));
template <int DT> struct LQuad;
template <> struct LQuad<H3D_F32> {
    static __device__ __forceinline__ f4 ld(const float *p) {
        const f4a4 v = *(const __attribute__((address_space(1))) f4a4 *)p;
        return f4{v[0], v[1], v[2], v[3]};
    }
};
template <> struct LQuad<H3D_BF16_SCALED> {
    static __device__ __forceinline__ f4 ld(const uint16_t *p) {
        const u2a2 w = *(const __attribute__((address_space(1))) u2a2 *)p;
        return f4{__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xffff0000u),
                  __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xffff0000u)};
    }
};

// a super-step: four K-steps of stage 1 (16 source rows); K-step i gives the
// lane of K slot q the row 16 S + 4 q + i, so a lane's factor values of the
// four K-steps are four consecutive rows of its column (one load)
template <int MT> struct LSlot {
    f4 a[MT];  // rows 16 S + 4 q .. + 3 of this lane's column of tile T
    f4 x[4];   // [i]: right-hand sides 4 r16 .. 4 r16 + 3 of row 16 S + 4 q + i
};

// ring depth in super-steps, U tiles loaded ahead, waves per SIMD
template <int MT> struct LfShape;
template <> struct LfShape<1> { static constexpr int D = 1, UP = 1, W = 3; };
template <> struct LfShape<2> { static constexpr int D = 2, UP = 2, W = 2; };
template <> struct LfShape<3> { static constexpr int D = 2, UP = 2, W = 1; };
template <> struct LfShape<4> { static constexpr int D = 2, UP = 2, W = 1; };

template <int DT, int MT>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LfShape<MT>::W)))
    k_leaf_fused(const int32_t *__restrict__ items, int64_t nitems, int64_t gbase,
                 const int32_t *__restrict__ leaf_off, const int64_t *__restrict__ grp_begin,
                 const int64_t *__restrict__ grp_blk,
                 void *const *__restrict__ uptr, void *const *__restrict__ vptr,
                 const int32_t *__restrict__ rank, const int32_t *__restrict__ soff,
                 const int32_t *__restrict__ slen, const float *__restrict__ scale2,
                 const float *__restrict__ Xs, int NP, double *__restrict__ Y) {
    using F = typename LFac<DT>::T;
    constexpr int D = LfShape<MT>::D, UP = LfShape<MT>::UP;
    const int64_t w = dev::xcd_run(blockIdx.x, gridDim.x);  // neighbouring leaves share sources
    if (w >= nitems)
        return;
    const int lane = threadIdx.x;
    const int r16 = lane & 15, q = lane >> 4;
    const int cs1 = 4 * (r16 & 3) + (r16 >> 2);  // this lane's factor column in a stage-1 tile
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
    struct Blk {
        int k, n;
        int64_t so;
        const F *V, *U;
        int64_t id;
    };
    auto load = [&](int64_t b) {
        const int64_t bj = grp_blk ? dev::cload(grp_blk + b) : b;
        return Blk{dev::cload(rank + bj), dev::cload(slen + bj), int64_t(dev::cload(soff + bj)),
                   static_cast<const F *>(dev::cload(vptr + bj)), static_cast<const F *>(dev::cload(uptr + bj)),
                   bj};
    };
    // stage-1 super-steps of a block padded to a multiple of D
    auto padded = [](int n) { return (((n + 15) >> 4) + D - 1) / D * D; };
    // first block of nonzero rank at or after b (e1 if none)
    auto skip = [&](int64_t b) {
        while (b < e1 && dev::cload(rank + (grp_blk ? dev::cload(grp_blk + b) : b)) <= 0)
            ++b;
        return b;
    };
    const int64_t bfirst = skip(e0);
    if (bfirst >= e1)
        return;  // no far block: Y keeps its rows
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        const bool lane_out = 4 * r16 < nv;
        // the leaf's rows of Y in FP64; each block's FP32 tiles are added
        // into them after the block
        double acc64[MT][4][4];
#pragma unroll
        for (int M = 0; M < MT; ++M)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int r = 16 * M + 4 * q + jj;
                const double *yp = Y + (bs + min(r, bm - 1)) * int64_t(NP) + bcol;
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    acc64[M][jj][N] = yp[N];
            }
        // refill cursor: block fb (metadata fc), padded step fs; the next
        // block's metadata in flight
        int64_t fb = bfirst;
        Blk fc = load(fb);
        int fS = padded(fc.n), fs = 0;
        int64_t fnb = skip(fb + 1);
        Blk fnx = fnb < e1 ? load(fnb) : fc;
        auto fadvance = [&] {
            if (++fs < fS)
                return;
            if (fnb >= e1) {  // past the last block: stay on its last step
                fs = fS - 1;
                return;
            }
            fb = fnb;
            fc = fnx;
            fS = padded(fc.n);
            fs = 0;
            fnb = skip(fb + 1);
            if (fnb < e1)
                fnx = load(fnb);
        };
        auto fill = [&](LSlot<MT> &R) {
            const int j0 = 16 * fs + 4 * q;
            const int ja = j0 < fc.n ? j0 : 0;  // a group wholly past the block: any rows
            // (a group reads at most three values past its column: the next
            // column, the next block or the chunk's 256 bytes of slack)
#pragma unroll
            for (int T = 0; T < MT; ++T)
                R.a[T] = LQuad<DT>::ld(fc.V + int64_t(min(16 * T + cs1, fc.k - 1)) * fc.n + ja);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                R.x[i] = *reinterpret_cast<const f4 *>(Xs + (fc.so + min(j0 + i, fc.n - 1)) * NP +
                                                       bcol);
        };
        LSlot<MT> R[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            fill(R[d]);
            fadvance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        int64_t cb = bfirst;
        Blk cc = fc;
        cc = load(cb);
        for (;;) {
            const int k = cc.k, n = cc.n;
            const int S1 = (n + 15) >> 4, S1p = padded(n), KT = (k + 15) >> 4;
            // U_b columns of the first UP tiles, needed after this block's stage 1
            float u[UP][4][MT];
#pragma unroll
            for (int T = 0; T < UP; ++T)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int M = 0; M < MT; ++M)
                        u[T][jj][M] =
                            LFac<DT>::ld(cc.U + int64_t(min(16 * T + 4 * jj + q, k - 1)) * bm + ic[M]);
            f4 C1[MT][4];
#pragma unroll
            for (int T = 0; T < MT; ++T)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    C1[T][N] = f4{0.f, 0.f, 0.f, 0.f};
            auto chunk = [&](int s0) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int s = s0 + d;
                    if (s < S1) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const bool aj = 16 * s + 4 * q + i < n;
                            float xv[4];
#pragma unroll
                            for (int N = 0; N < 4; ++N)
                                xv[N] = aj ? R[d].x[i][N] : 0.f;
#pragma unroll
                            for (int T = 0; T < MT; ++T)
                                if (T < KT)
#pragma unroll
                                    for (int N = 0; N < 4; ++N)
                                        C1[T][N] = mma(R[d].a[T][i], xv[N], C1[T][N]);
                        }
                    }
                    fill(R[d]);
                    fadvance();
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            // the first chunk on its own: its waits then count the U loads
            // just issued (a shared loop header would count them as absent
            // and wait for most of the ring at every block)
            chunk(0);
            for (int s0 = D; s0 < S1p; s0 += D)
                chunk(s0);
            if constexpr (DT == H3D_BF16_SCALED) {
                const float sc = scale2[2 * cc.id] * scale2[2 * cc.id + 1];
#pragma unroll
                for (int T = 0; T < MT; ++T)
#pragma unroll
                    for (int N = 0; N < 4; ++N)
                        C1[T][N] *= sc;
            }
            // ---- stage 2: C2[M][N] = U[16 M .., 16 T + 4 jj + q] C1[T][N][jj]
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
                float ut[4][MT];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                    for (int M = 0; M < MT; ++M) {
                        if (T < UP)
                            ut[jj][M] = u[T < UP ? T : 0][jj][M];
                        else
                            ut[jj][M] = LFac<DT>::ld(
                                cc.U + int64_t(min(16 * T + 4 * jj + q, k - 1)) * bm + ic[M]);
                    }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (16 * T + 4 * jj >= k)
                        break;  // columns 16 T + 4 jj .. all past the rank
                    const bool kc = 16 * T + 4 * jj + q < k;
#pragma unroll
                    for (int M = 0; M < MT; ++M) {
                        const float av = (kc && ai[M]) ? ut[jj][M] : 0.f;
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
                        acc64[M][jj][N] += double(C2[M][N][jj]);
            cb = skip(cb + 1);
            if (cb >= e1)
                break;
            cc = load(cb);
        }
        if (lane_out) {
#pragma unroll
            for (int M = 0; M < MT; ++M)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = 16 * M + 4 * q + jj;
                    if (r < bm) {
                        double *yp = Y + (bs + r) * int64_t(NP) + nb + 4 * r16;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            yp[N] = acc64[M][jj][N];
                    }
                }
        }
    }
}

// Many right-hand sides, near field with FP32 entries (the FP32 and BF16
// factor forms): one wave per target leaf of at most 16 MT rows, all its row
// tiles at once, so that every fragment of x is loaded once for the leaf (one
// wave per 16-row tile read the rows of x of all the leaf's near leaves once
// per tile).  A K-step takes four source points of a near leaf (K slot q =
// point j0 + q); a lane evaluates the entries of its MT target rows against
// its source point in FP32 (distances formed in FP64 and rounded once), and
// its four x values of the point are one 16-byte load (tile N, column n is
// right-hand side 4 n + N).  Entries of rows past the leaf, of source points
// past the near leaf and of a point with itself are zero.  The FP32 sums of
// a row run in the same order as in the one-tile-per-wave form.  The loads of
// the next two K-steps are in flight while a step's MFMAs run (a cursor over
// the near leaves' K-steps in list order, with the steady part and tail of
// the other rings).
struct NSlot {
    double xj, yj, zj;  // this lane's source point
    int64_t gj;
    bool ok;            // the point lies inside its near leaf
    f4 xv;              // its right-hand sides 4 r16 .. 4 r16 + 3
};

template <int MT, int KIND>
__global__ void __launch_bounds__(256)
    k_near_leaf(const int32_t *__restrict__ items, int64_t nitems,
                const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ near_ptr,
                const int32_t *__restrict__ near_s, const double *__restrict__ px,
                const double *__restrict__ py, const double *__restrict__ pz, int kind, float kp,
                const float *__restrict__ Xs, int NP, double *__restrict__ Y) {
    const int64_t w = dev::xcd_run(blockIdx.x, gridDim.x) * 4 +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nitems)
        return;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    const int64_t t = dev::cload(items + w);
    const int32_t t0 = dev::cload(leaf_off + t), m = dev::cload(leaf_off + t + 1) - t0;
    const int e0 = dev::cload(near_ptr + t), e1 = dev::cload(near_ptr + t + 1);
    double xi[MT], yi[MT], zi[MT];
    int64_t gi[MT];
    bool ai[MT];
#pragma unroll
    for (int T = 0; T < MT; ++T) {
        const int i = 16 * T + r16;
        ai[T] = i < m;
        gi[T] = t0 + (ai[T] ? i : 0);
        xi[T] = px[gi[T]];
        yi[T] = py[gi[T]];
        zi[T] = pz[gi[T]];
    }
    int S = 0;  // K-steps of four source points over the near leaves
    for (int e = e0; e < e1; ++e) {
        const int32_t sl = dev::cload(near_s + e);
        S += (dev::cload(leaf_off + sl + 1) - dev::cload(leaf_off + sl) + 3) >> 2;
    }
    if (S == 0)
        return;
    for (int nb = 0; nb < NP; nb += 64) {
        const int nv = min(64, NP - nb);
        const int bcol = nb + 4 * min(r16, nv / 4 - 1);
        f4 acc[MT][4];
#pragma unroll
        for (int T = 0; T < MT; ++T)
#pragma unroll
            for (int N = 0; N < 4; ++N)
                acc[T][N] = f4{0.f, 0.f, 0.f, 0.f};
        // refill cursor over the K-steps of the near leaves in list order,
        // two steps in flight; past the last step it stays there (never
        // consumed)
        int fe = e0, fj = 0;
        int32_t fs0 = 0, fns = 1;
        auto leaf_rows = [&](int e) {
            const int32_t sl = dev::cload(near_s + e);
            fs0 = dev::cload(leaf_off + sl);
            fns = dev::cload(leaf_off + sl + 1) - fs0;
        };
        leaf_rows(fe);
        auto fill = [&](NSlot &R) {
            const int j = fj + q;
            R.gj = fs0 + min(j, fns - 1);
            R.ok = j < fns;
            R.xj = px[R.gj];
            R.yj = py[R.gj];
            R.zj = pz[R.gj];
            R.xv = *reinterpret_cast<const f4 *>(Xs + R.gj * NP + bcol);
        };
        auto advance = [&] {
            if ((fj += 4) < fns)
                return;
            if (fe + 1 >= e1) {  // past the last step: stay on it
                fj -= 4;
                return;
            }
            fj = 0;
            leaf_rows(++fe);
        };
        auto step = [&](const NSlot &R) {
            float a[MT];
#pragma unroll
            for (int T = 0; T < MT; ++T) {
                const double dx = xi[T] - R.xj, dy = yi[T] - R.yj, dz = zi[T] - R.zj;
                const float r2 = float(dx * dx + dy * dy + dz * dz);
                a[T] = (ai[T] && R.ok && R.gj != gi[T])
                           ? dev::kernel_f32(KIND >= 0 ? KIND : kind, kp, r2)
                           : 0.f;
            }
#pragma unroll
            for (int T = 0; T < MT; ++T)
#pragma unroll
                for (int N = 0; N < 4; ++N)
                    acc[T][N] = mma(a[T], R.xv[N], acc[T][N]);
        };
        NSlot R[2];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            fill(R[d]);
            advance();
            __builtin_amdgcn_sched_barrier(0);  // slots in order (the waits count on it)
        }
        int s0 = 0;
        for (; s0 + 2 <= S; s0 += 2) {
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                step(R[d]);
                fill(R[d]);
                advance();
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (s0 < S)
            step(R[0]);
        if (4 * r16 < nv) {
#pragma unroll
            for (int T = 0; T < MT; ++T)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int r = 16 * T + 4 * q + jj;
                    if (r < m) {
                        double *yp = Y + (t0 + r) * int64_t(NP) + nb + 4 * r16;
#pragma unroll
                        for (int N = 0; N < 4; ++N)
                            yp[N] = double(acc[T][N][jj]);
                    }
                }
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

void launch_leaf_fused(Plan &P, const float *Xs, int NP, double *Y, bool adjoint, hipStream_t s) {
    const int l = P.L;
    // the adjoint: blocks taken by source leaf, U and V exchanged, the rows of
    // stage 1 in the target leaf
    const int64_t *gblk = adjoint ? P.src_blk : nullptr;
    void *const *p1 = adjoint ? P.blk_uptr : P.blk_vptr;  // stage-1 factor (K over its rows)
    void *const *p2 = adjoint ? P.blk_vptr : P.blk_uptr;  // stage-2 factor (the leaf's rows)
    const int32_t *off1 = adjoint ? P.blk_toff : P.blk_soff;
    const int32_t *len1 = adjoint ? P.blk_m : P.blk_n;
#define H3D_LF(DT, MT)                                                                          \
    k_leaf_fused<DT, MT><<<int(P.lf_n[MT - 1]), 64, 0, s>>>(                                    \
        P.lf_items[MT - 1], P.lf_n[MT - 1], P.box_base[l], P.leaf_off, P.tgt_begin, gblk, p2,    \
        p1, P.blk_rank, off1, len1, P.blk_scale, Xs, NP, Y)
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

// The near field of a many-RHS product with FP32 entries, one wave per leaf
// (false when the leaf classes do not apply: some leaf holds more than 64
// rows).
bool launch_near_leaves(Plan &P, const float *Xs, int NP, double *Y, hipStream_t s) {
    if (P.L < 1 || !leaf_fused_tables(P, s))
        return false;
    const float kp = float(P.cfg.kernel_param);
    // the Laplace kernel has launches of its own (the general ones carry
    // every kernel's formula)
    const bool lap = P.cfg.kernel == H3D_LAPLACE;
#define H3D_NL(MT, K)                                                                           \
    k_near_leaf<MT, K><<<int((P.lf_n[MT - 1] + 3) / 4), 256, 0, s>>>(                          \
        P.lf_items[MT - 1], P.lf_n[MT - 1], P.leaf_off, P.near_ptr, P.near_s, P.px, P.py, P.pz, \
        P.cfg.kernel, kp, Xs, NP, Y)
#define H3D_NLK(MT)                                                                             \
    if (lap)                                                                                    \
        H3D_NL(MT, H3D_LAPLACE);                                                                \
    else                                                                                        \
        H3D_NL(MT, -1);
    for (int mt = 1; mt <= 4; ++mt) {
        if (P.lf_n[mt - 1] == 0)
            continue;
        switch (mt) {
        case 1: H3D_NLK(1) break;
        case 2: H3D_NLK(2) break;
        case 3: H3D_NLK(3) break;
        default: H3D_NLK(4) break;
        }
        H3D_LAUNCH_CHECK();
    }
#undef H3D_NLK
#undef H3D_NL
    return true;
}

}  // namespace h3d
