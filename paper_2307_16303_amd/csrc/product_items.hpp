// Per-item device code of the mat-vec (Algorithm 2): the gather of one row,
// the near field of one leaf and stage 2 of one chunk box (stage-1 work items:
// stage1_items.hpp).  The per-phase kernels of a single operator and the
// phase launches of a batch of operators both call these functions, so a
// problem computes the same sums in either form.
#pragma once

#include "h3d_internal.hpp"

namespace h3d {
namespace dev {

// Workgroups are dealt to the eight XCDs in turn, each XCD with its own L2.
// Renumbering workgroup b as below gives every XCD a contiguous run of the
// grid (XCD x takes q or q + 1 consecutive numbers), so neighbouring work
// items, which share inputs, meet in one L2.  A bijection on [0, nwg).
__device__ __forceinline__ int64_t xcd_run(int64_t b, int64_t nwg) {
    const int64_t q = nwg >> 3, r = nwg & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// The grid dealt to the XCDs in chunks of C consecutive workgroups in turn
// (chunk j to XCD j mod 8): where the cost of an item changes along the grid,
// as over the problems of a batch, every XCD still gets an even share, and
// neighbouring items still meet in one L2.  The workgroups past the last whole
// round of 8 C chunks are split as by xcd_run; C = 0 is xcd_run itself.
template <int C> __device__ __forceinline__ int64_t xcd_chunks(int64_t b, int64_t nwg) {
    if constexpr (C == 0) {
        return xcd_run(b, nwg);
    } else {
        const int64_t round = 8 * C, full = nwg / round;
        if (b < full * round) {
            const int64_t x = b & 7, k = b >> 3;  // the k-th workgroup of XCD x
            return ((k / C) * 8 + x) * C + k % C;
        }
        return full * round + xcd_run(b - full * round, nwg - full * round);
    }
}

// A load from a table that no wave writes during the kernel: through the
// constant address space it stays a scalar load when the index is uniform,
// also after the kernel's own global stores or atomics.
template <typename T> __device__ __forceinline__ T cload(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// Factor loads.  Plain loads keep the lines in L2: a column slice rarely
// starts on a 128-byte line, and the part of a line that the next slice
// needs is then still cached (with the non-temporal hint such lines were
// fetched twice).  kS2NonTemporal selects the hint for the stage-2 stream.
constexpr bool kS2NonTemporal = false;

template <int DT> struct Fac;
template <> struct Fac<H3D_F64> {
    using T = double;
    static __device__ __forceinline__ double cvt(T v) { return v; }
};
template <> struct Fac<H3D_F32> {
    using T = float;
    static __device__ __forceinline__ double cvt(T v) { return double(v); }
};
template <> struct Fac<H3D_BF16_SCALED> {
    using T = uint16_t;
    static __device__ __forceinline__ double cvt(T v) {
        return double(__uint_as_float(uint32_t(v) << 16));
    }
};
// Factor pointers come from tables in memory, where the compiler cannot see
// that they address global memory: without the address space every factor
// load would be a flat load, which also waits on the LDS/scalar counter.
template <int DT, bool NT = false>
__device__ __forceinline__ typename Fac<DT>::T fac_raw(const typename Fac<DT>::T *p) {
    using G = const __attribute__((address_space(1))) typename Fac<DT>::T;
    if constexpr (NT)
        return __builtin_nontemporal_load((G *)p);
    else
        return *(G *)p;
}
// p as a pointer to global memory: accesses through it compile to global
// loads and stores.  (A pointer read from device memory, as from a batch's
// descriptors, is otherwise accessed with flat instructions, which also count
// against the scalar and LDS counter and cost registers.)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *glob(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
template <int DT, bool NT = false>
__device__ __forceinline__ double fac_ld(const typename Fac<DT>::T *p) {
    return Fac<DT>::cvt(fac_raw<DT, NT>(p));
}

__device__ __forceinline__ double kernel_f(int kind, double kp, double r) {
    if (r == 0.0)
        return 0.0;
    switch (kind) {
    case H3D_LAPLACE:
        return 1.0 / (4.0 * 3.14159265358979323846 * r);
    case H3D_YUKAWA:
        return exp(-kp * r) / r;
    case H3D_INV_R4: {
        double r2 = r * r;
        return 1.0 / (r2 * r2);
    }
    case H3D_COS_R:
        return cos(kp * r) / r;
    default:
        return 0.0;
    }
}

// Kernel entry in FP32 from the squared distance (the FP32 and BF16 forms):
// one reciprocal square root; 0 at r = 0.  The squared distance comes from
// FP64 coordinate differences, so it is symmetric in the two points.
__device__ __forceinline__ float kernel_f32(int kind, float kp, float r2) {
    if (r2 == 0.0f)
        return 0.0f;
    const float ir = __frsqrt_rn(r2);
    switch (kind) {
    case H3D_LAPLACE:
        return ir * 0.0795774715459476679f;  // 1/(4 pi)
    case H3D_YUKAWA:
        return __expf(-kp * r2 * ir) * ir;
    case H3D_INV_R4:
        return ir * ir * ir * ir;
    case H3D_COS_R:
        return __cosf(kp * r2 * ir) * ir;
    default:
        return 0.0f;
    }
}

// ---------------------------------------------------------------------------
// xp[:, p] = x[perm[p], :] for one sorted row p < n
__device__ __forceinline__ void gather_row(const void *__restrict__ x, int io_f32, int64_t ldx,
                                           int64_t n, int nrhs, const int32_t *__restrict__ perm,
                                           double *__restrict__ xp, int64_t p) {
    const int64_t src = glob(perm)[p];
    for (int q = 0; q < nrhs; ++q) {
        double v = io_f32 ? double(glob(static_cast<const float *>(x))[q * ldx + src])
                          : glob(static_cast<const double *>(x))[q * ldx + src];
        glob(xp)[q * n + p] = v;
    }
}

// ---------------------------------------------------------------------------
// near field: one wave per leaf; lane = (row within a pass of R rows, source
// slice q of Q = 64/R).  The sources of the whole near list, concatenated in
// list order, are staged through LDS in chunks of kChunk points: one pass of
// loads per chunk (a leaf's near list of up to 19 leaves of a few points is
// one chunk), every lane finding the list entry of each point it stages by a
// binary search over the entries' first positions.
constexpr int kChunk = 128;

// E32: kernel entries evaluated in FP32 (forms with FP32 or BF16 factors),
// accumulated in FP64.  KIND >= 0 fixes the kernel at compile time (only its
// formula is inlined into the loop); -1 takes `kind`.
template <int NR, bool E32 = false, int KIND = -1>
__device__ __forceinline__ void near_leaf(int64_t t, const int32_t *__restrict__ leaf_off_,
                                          const int32_t *__restrict__ near_ptr_,
                                          const int32_t *__restrict__ near_s_,
                                          const double *__restrict__ px_,
                                          const double *__restrict__ py_,
                                          const double *__restrict__ pz_, int kind, double kp,
                                          int nrhs, const double *__restrict__ xp_, int64_t n,
                                          double *__restrict__ yn_) {
    // global-typed pointers (glob): the batch reads them from device memory
    const auto leaf_off = glob(leaf_off_), near_ptr = glob(near_ptr_), near_s = glob(near_s_);
    const auto px = glob(px_), py = glob(py_), pz = glob(pz_);
    const auto xp = glob(xp_);
    const auto yn = glob(yn_);
    __shared__ double sx[kChunk], sy[kChunk], sz[kChunk];
    __shared__ double sv[NR][kChunk];
    __shared__ int32_t sg[kChunk];        // sorted index of each staged source
    __shared__ int32_t s_beg[64], s_row[64];  // per list entry: first position, first row
    const int lane = threadIdx.x;
    const int kd = KIND >= 0 ? KIND : kind;
    const int32_t t0 = leaf_off[t];
    const int m = leaf_off[t + 1] - t0;
    if (m == 0)
        return;
    int R = 1;
    while (R < m && R < 64)
        R <<= 1;
    const int Q = 64 / R;
    const int e0 = near_ptr[t], e1 = near_ptr[t + 1];
    for (int rowb = 0; rowb < m; rowb += R) {
        const int i = rowb + (lane % R);
        const int q = lane / R;
        const bool ai = i < m;
        const int64_t gi = t0 + (ai ? i : 0);
        const double xi = px[gi], yi = py[gi], zi = pz[gi];
        for (int rb = 0; rb < nrhs; rb += NR) {
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = 0.0;
            // the list, 64 entries at a time
            for (int ea = e0; ea < e1; ea += 64) {
                const int ne = min(64, e1 - ea);
                int row0 = 0, ns = 0;
                if (lane < ne) {
                    const int32_t s = near_s[ea + lane];
                    row0 = leaf_off[s];
                    ns = leaf_off[s + 1] - row0;
                }
                int incl = ns;  // inclusive prefix sum of the sizes over the lanes
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int v = __shfl_up(incl, d, 64);
                    if (lane >= d)
                        incl += v;
                }
                const int total = __shfl(incl, ne - 1, 64);
                __syncthreads();  // the previous chunk's readers are done
                if (lane < ne) {
                    s_beg[lane] = incl - ns;
                    s_row[lane] = row0;
                }
                for (int cb = 0; cb < total; cb += kChunk) {
                    const int cn = min(kChunk, total - cb);
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < kChunk / 64; ++u) {
                        const int f = cb + u * 64 + lane;
                        if (f < cb + cn) {
                            // last entry whose first position is <= f (entries
                            // of empty leaves share the next entry's position)
                            int lo = 0, hi = ne;
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (s_beg[mid] <= f)
                                    lo = mid;
                                else
                                    hi = mid;
                            }
                            const int32_t gj = s_row[lo] + (f - s_beg[lo]);
                            const int jj = f - cb;
                            sg[jj] = gj;
                            sx[jj] = px[gj];
                            sy[jj] = py[gj];
                            sz[jj] = pz[gj];
#pragma unroll
                            for (int c = 0; c < NR; ++c)
                                sv[c][jj] = (rb + c < nrhs) ? xp[(rb + c) * n + gj] : 0.0;
                        }
                    }
                    __syncthreads();
                    if (ai) {
                        for (int j = q; j < cn; j += Q) {
                            if (sg[j] == gi)
                                continue;
                            const double dx = xi - sx[j], dy = yi - sy[j], dz = zi - sz[j];
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            const double f = E32 ? double(kernel_f32(kd, float(kp), float(r2)))
                                                 : kernel_f(kd, kp, sqrt(r2));
#pragma unroll
                            for (int c = 0; c < NR; ++c)
                                acc[c] += f * sv[c][j];
                        }
                    }
                }
            }
            for (int off = R; off < 64; off <<= 1)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    acc[c] += __shfl_xor(acc[c], off, 64);
            if (ai && q == 0)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (rb + c < nrhs)
                        yn[(rb + c) * n + gi] = acc[c];
        }
    }
}

// ---------------------------------------------------------------------------
// stage 2: one workgroup per box of the chunk level, one lane per row (two
// for boxes of 65..128 rows).  At levels up to the chunk level every lane of
// the workgroup lies in the same box, so the block metadata and z are
// wave-uniform (scalar loads) and each lane streams one column slice of U per
// load, U2 loads in flight; the waves split the box's blocks.
struct S2Tab {
    int64_t box_base[kMaxLevels + 1];
    int L, lc;
    int panel;  // the factors streamed are U_b stored as row panels above lc
};

template <int DT, int NR, int U2>
__device__ __forceinline__ void stage2_block(const typename Fac<DT>::T *__restrict__ p, int bm, int k,
                                             const double *__restrict__ zz, int64_t ldz, int rb,
                                             int nrhs, double (&acc)[NR]) {
    // raw values in flight (one register each for FP32/BF16), converted at use
    using T = typename Fac<DT>::T;
    int c = 0;
    for (; c + U2 <= k; c += U2) {
        T v[U2];
#pragma unroll
        for (int u = 0; u < U2; ++u)
            v[u] = fac_raw<DT, kS2NonTemporal>(p + int64_t(c + u) * bm);
#pragma unroll
        for (int u = 0; u < U2; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (NR == 1 || rb + q < nrhs)
                    acc[q] += Fac<DT>::cvt(v[u]) * glob(zz)[(rb + q) * ldz + c + u];
    }
    for (; c < k; ++c) {
        const double v = fac_ld<DT, kS2NonTemporal>(p + int64_t(c) * bm);
#pragma unroll
        for (int q = 0; q < NR; ++q)
            if (NR == 1 || rb + q < nrhs)
                acc[q] += v * glob(zz)[(rb + q) * ldz + c];
    }
}

// The same for two rows per lane, d rows apart (d = 0 for a lane whose second
// row lies past the box: it then repeats its first load and drops the sum).
template <int DT, int NR, int U2>
__device__ __forceinline__ void stage2_block2(const typename Fac<DT>::T *__restrict__ p, int d,
                                              int bm, int k, const double *__restrict__ zz,
                                              int64_t ldz, int rb, int nrhs, double (&a0)[NR],
                                              double (&a1)[NR]) {
    using T = typename Fac<DT>::T;
    int c = 0;
    for (; c + U2 <= k; c += U2) {
        T v[U2], w[U2];
#pragma unroll
        for (int u = 0; u < U2; ++u) {
            v[u] = fac_raw<DT, kS2NonTemporal>(p + int64_t(c + u) * bm);
            w[u] = fac_raw<DT, kS2NonTemporal>(p + d + int64_t(c + u) * bm);
        }
#pragma unroll
        for (int u = 0; u < U2; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (NR == 1 || rb + q < nrhs) {
                    const double zq = glob(zz)[(rb + q) * ldz + c + u];
                    a0[q] += Fac<DT>::cvt(v[u]) * zq;
                    a1[q] += Fac<DT>::cvt(w[u]) * zq;
                }
    }
    for (; c < k; ++c) {
        const double v = fac_ld<DT, kS2NonTemporal>(p + int64_t(c) * bm);
        const double w = fac_ld<DT, kS2NonTemporal>(p + d + int64_t(c) * bm);
#pragma unroll
        for (int q = 0; q < NR; ++q)
            if (NR == 1 || rb + q < nrhs) {
                const double zq = glob(zz)[(rb + q) * ldz + c];
                a0[q] += v * zq;
                a1[q] += w * zq;
            }
    }
}

template <int DT, int NR, int kS2Waves>
__device__ __forceinline__ void
    stage2_chunk(int64_t B, const S2Tab &tab, const int32_t *__restrict__ leaf_off_,
                 const int32_t *__restrict__ leaf_of_, const int64_t *__restrict__ grp_begin_,
                 const int64_t *__restrict__ grp_blk_, void *const *__restrict__ fptr_,
                 const int32_t *__restrict__ rank_, const int64_t *__restrict__ blk_col0_,
                 const double *__restrict__ z, int64_t ldz, const double *yn_, int64_t n, int nrhs,
                 const int32_t *__restrict__ perm_, void *__restrict__ yout, int64_t ldy,
                 int io_f32, int lb, int le, double *ypart) {
    using T = typename Fac<DT>::T;
    // the tables as pointers to global memory (glob), also when they were
    // read from device memory
    const auto leaf_off = glob(leaf_off_), leaf_of = glob(leaf_of_);
    const auto grp_begin = glob(grp_begin_), grp_blk = glob(grp_blk_);
    const auto fptr = glob(fptr_);
    const auto rank = glob(rank_);
    const auto blk_col0 = glob(blk_col0_);
    const auto yn = glob(yn_);
    const auto perm = glob(perm_);
    __shared__ double part[kS2Waves][NR][64];
    const int L = tab.L, lc = tab.lc;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int shc = 3 * (L - lc);
    const int32_t r0 = leaf_off[B << shc], r1 = leaf_off[(B + 1) << shc];
    // Passes of up to 128 rows: a box of 65..128 rows reads every coarse
    // column slice in one pass, two rows per lane (rows rowb + lane and
    // rowb + 64 + lane), instead of a second pass over the same columns.
    for (int32_t rowb = r0; rowb < r1;) {
        const bool two = r1 - rowb > 64;
        const int32_t rowA = rowb + lane, rowB = rowb + 64 + lane;
        const bool actA = rowA < r1, actB = two && rowB < r1;
        const int32_t rrA = actA ? rowA : r0;
        const int dB = actB ? 64 : 0;
        for (int rb = 0; rb < nrhs; rb += NR) {
            double acc[2][NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const bool ok = wv == 0 && (NR == 1 || rb + c < nrhs);
                acc[0][c] = ok ? yn[(rb + c) * n + rrA] : 0.0;
                acc[1][c] = (ok && two) ? yn[(rb + c) * n + rrA + dB] : 0.0;
            }
            // levels whose boxes contain the whole chunk box: wave-uniform;
            // the waves of the workgroup take every kS2Waves-th block
            for (int l = lb; l <= min(lc, le); ++l) {
                const int sh = 3 * (L - l);
                const int64_t t = B >> (3 * (lc - l));
                const int64_t g = tab.box_base[l] + t;
                const int32_t bs = leaf_off[t << sh];
                const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                // this chunk box's panel of U_b: rows r0..r1, leading dimension r1 - r0
                const bool pan = tab.panel && l < lc;
                const int32_t ld = pan ? r1 - r0 : bm;
                const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                for (int64_t e = e0 + wv; e < e1; e += kS2Waves) {
                    const int64_t bi = grp_blk ? grp_blk[e] : e;
                    const int kb = rank[bi];
                    const T *p = static_cast<const T *>(fptr[bi]) +
                                 (pan ? int64_t(r0 - bs) * kb + (rrA - r0) : int64_t(rrA - bs));
                    if (two)
                        stage2_block2<DT, NR, 8>(p, dB, ld, kb, z + blk_col0[bi],
                                                                  ldz, rb, nrhs, acc[0], acc[1]);
                    else
                        stage2_block<DT, NR, 8>(p, ld, kb, z + blk_col0[bi], ldz,
                                                                 rb, nrhs, acc[0]);
                }
            }
            // finer levels and the output, per row of the lane: a constant row
            // slot, so that the accumulators stay in registers
            auto finish = [&](const int h, double (&ah)[NR]) {
                const int32_t row = h ? rowB : rowA;
                const bool act = h ? actB : actA;
                const int32_t rr = act ? row : r0;
                const int32_t leaf = leaf_of[rr];
                // finer levels: every lane follows the box of its own row
                for (int l = max(lc + 1, lb); l <= le; ++l) {
                    const int sh = 3 * (L - l);
                    const int64_t t = int64_t(leaf) >> sh;
                    const int64_t g = tab.box_base[l] + t;
                    const int32_t bs = leaf_off[t << sh];
                    const int32_t bm = leaf_off[(t + 1) << sh] - bs;
                    const int32_t loc = rr - bs;
                    const int64_t e0 = grp_begin[g], e1 = grp_begin[g + 1];
                    if (grp_blk) {
                        for (int64_t e = e0 + wv; e < e1; e += kS2Waves) {
                            const int64_t bi = grp_blk[e];
                            const T *p = static_cast<const T *>(fptr[bi]) + loc;
                            stage2_block<DT, NR, 4>(p, bm, rank[bi], z + blk_col0[bi], ldz, rb,
                                                          nrhs, ah);
                        }
                    } else if (e1 > e0) {
                        // The blocks of a target box are consecutive, and so are their
                        // z columns: wave wv takes columns [cb, ce) of the box's K.
                        // When the U_b also lie back to back (one ACA batch), they form
                        // one bm x K matrix, streamed as such; otherwise the same column
                        // range is walked block by block, so that the sums, and their
                        // order, do not depend on how the factors were batched.
                        const int64_t zc0 = blk_col0[e0];
                        const int kt = int(blk_col0[e1] - zc0);
                        const int cb = (kt * wv) / kS2Waves, ce = (kt * (wv + 1)) / kS2Waves;
                        const T *pf = static_cast<const T *>(fptr[e0]);
                        const T *pl = static_cast<const T *>(fptr[e1 - 1]);
                        if (pl + int64_t(bm) * rank[e1 - 1] == pf + int64_t(bm) * kt) {
                            stage2_block<DT, NR, 8>(pf + loc + int64_t(cb) * bm, bm, ce - cb,
                                                          z + zc0 + cb, ldz, rb, nrhs, ah);
                        } else {
                            for (int64_t e = e0; e < e1; ++e) {
                                const int c0 = int(blk_col0[e] - zc0);
                                if (c0 >= ce)
                                    break;
                                const int lo = max(cb, c0), hi = min(ce, c0 + rank[e]);
                                if (lo < hi)
                                    stage2_block<DT, NR, 8>(
                                        static_cast<const T *>(fptr[e]) + loc +
                                            int64_t(lo - c0) * bm,
                                        bm, hi - lo, z + zc0 + lo, ldz, rb, nrhs, ah);
                            }
                        }
                    }
                }
                // combine the waves' partial sums in a fixed order
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    part[wv][q][lane] = ah[q];
                __syncthreads();
                if (wv == 0) {
                    double y[NR];
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        double v = part[0][q][lane];
#pragma unroll
                        for (int w2 = 1; w2 < kS2Waves; ++w2)
                            v += part[w2][q][lane];
                        y[q] = v;
                    }
                    if (act && ypart) {
                        // partial sums in sorted order (level-by-level profiling)
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < nrhs)
                                glob(ypart)[(rb + q) * n + row] = y[q];
                    } else if (act) {
                        const int64_t dst = perm[row];
#pragma unroll
                        for (int q = 0; q < NR; ++q)
                            if (NR == 1 || rb + q < nrhs) {
                                if (io_f32)
                                    glob(static_cast<float *>(yout))[(rb + q) * ldy + dst] = float(y[q]);
                                else
                                    glob(static_cast<double *>(yout))[(rb + q) * ldy + dst] = y[q];
                            }
                    }
                }
                __syncthreads();
            };
            finish(0, acc[0]);
            if (two)
                finish(1, acc[1]);
        }
        rowb += two ? 128 : 64;
    }
}

}  // namespace dev
}  // namespace h3d
