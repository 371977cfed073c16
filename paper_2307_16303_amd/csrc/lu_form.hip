// The paper's storage form of the low-rank blocks (Sec. 4.1, eqs. (prank) and
// (LR); the low-rank step of Algorithm 2).  A block K(X,Y) keeps only its ACA
// pivots sigma (rows of X) and tau (columns of Y) and the LU factors of
// K(sigma, tau); every product regenerates the kernel entries of K(sigma, Y)
// and K(X, tau) and applies
//     y(X) += K(X, tau) R^-1 L^-1 K(sigma, Y) x(Y),
// so the factor streams of the explicit form become kernel evaluations: the
// product is bound by the vector ALUs, and the stored data shrinks from
// (m + n) k to k^2 + 2k values per block.
//
// Build: the LU factors are read off the FP64 ACA factors at the pivots (L
// from U on the pivot rows, the unit-diagonal R from V on the pivot columns;
// both vanish on the earlier pivots), packed into one k x k column-major
// matrix per block (L on and below the diagonal, R above it).  Every factor
// column g (block b, pivot c, g = col0_b + c) records the sorted rows of its
// two pivot points.
//
// Product (forward; the adjoint exchanges the roles of X, sigma, L and Y, tau,
// R^T):
//   stage 1  one wave per block (or per part of a block whose source side is
//            longer than kLuPart): w = K(sigma, Y) x(Y) with the sources
//            staged through LDS, lanes = (pivot, source slice); then the two
//            triangular solves in registers (lane r holds row r), z_b = w.
//   stage 2  one wave per leaf: for every level, the factor columns of the
//            blocks whose target contains the leaf form one contiguous range
//            (blocks of a target box are consecutive); the pivot points and
//            z values of that range are staged through LDS and every row of
//            the leaf sums K(x_i, y_tau) z over them, added to the near-field
//            sums and written out in the caller's point order.
#include "product_items.hpp"

namespace h3d {

namespace {

constexpr int kLuChunk = 128;  // points / columns staged per LDS pass
constexpr int kLuPart = 4096;  // source rows per stage-1 work item
constexpr int kLuNR = kLuGroup;  // right-hand sides per pass of the many-column kernels

struct LuItem {
    int32_t b;     // block
    int32_t part;  // -1: the whole source side, then the solve; else part index
    int64_t wo;    // part items: first partial column (parts of a block are consecutive)
};

struct LuSplit {
    int32_t b, np;
    int64_t wo;  // partial column of part 0
};

template <int KIND>
__device__ __forceinline__ double entry(int kind, double kp, double dx, double dy, double dz) {
    return dev::kernel_f(KIND >= 0 ? KIND : kind, kp, sqrt(dx * dx + dy * dy + dz * dz));
}

// value of slot pc (wave-uniform) of a per-lane register array, from lane lc
template <int NR>
__device__ __forceinline__ void bcast(const double (&w)[kLuSlots][NR], int pc, int lc,
                                      double (&o)[NR]) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        double v = w[0][c];
#pragma unroll
        for (int p = 1; p < kLuSlots; ++p)
            if (pc == p)
                v = w[p][c];
        o[c] = __shfl(v, lc, 64);
    }
}

// In-register triangular solves of one block: lane l holds row p 64 + l in
// slot p.  Forward product: w <- R^-1 L^-1 w; adjoint: w <- L^-T R^-T w.
template <int NR>
__device__ __forceinline__ void lu_solve(const double *__restrict__ lu, int k, bool adjoint,
                                         double (&w)[kLuSlots][NR]) {
    const int lane = threadIdx.x;
    using G = const __attribute__((address_space(1))) double;
    const G *A = (const G *)lu;
    double wc[NR];
    if (!adjoint) {
        // L: column c below the diagonal
        for (int c = 0; c < k; ++c) {
            bcast<NR>(w, c >> 6, c & 63, wc);
            const double d = A[int64_t(c) * k + c];
#pragma unroll
            for (int q = 0; q < NR; ++q)
                wc[q] = wc[q] / d;
#pragma unroll
            for (int p = 0; p < kLuSlots; ++p) {
                const int r = p * 64 + lane;
                if (r == c) {
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        w[p][q] = wc[q];
                } else if (r > c && r < k) {
                    const double a = A[int64_t(c) * k + r];
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        w[p][q] -= a * wc[q];
                }
            }
        }
        // R (unit diagonal): column c above the diagonal
        for (int c = k - 1; c > 0; --c) {
            bcast<NR>(w, c >> 6, c & 63, wc);
#pragma unroll
            for (int p = 0; p < kLuSlots; ++p) {
                const int r = p * 64 + lane;
                if (r < c) {
                    const double a = A[int64_t(c) * k + r];
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        w[p][q] -= a * wc[q];
                }
            }
        }
    } else {
        // R^T (unit lower): R^T[r][c] = R[c][r], stored at (row c, column r)
        for (int c = 0; c + 1 < k; ++c) {
            bcast<NR>(w, c >> 6, c & 63, wc);
#pragma unroll
            for (int p = 0; p < kLuSlots; ++p) {
                const int r = p * 64 + lane;
                if (r > c && r < k) {
                    const double a = A[int64_t(r) * k + c];
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        w[p][q] -= a * wc[q];
                }
            }
        }
        // L^T (upper): L^T[r][c] = L[c][r], stored at (row c, column r)
        for (int c = k - 1; c >= 0; --c) {
            bcast<NR>(w, c >> 6, c & 63, wc);
            const double d = A[int64_t(c) * k + c];
#pragma unroll
            for (int q = 0; q < NR; ++q)
                wc[q] = wc[q] / d;
#pragma unroll
            for (int p = 0; p < kLuSlots; ++p) {
                const int r = p * 64 + lane;
                if (r == c) {
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        w[p][q] = wc[q];
                } else if (r < c) {
                    const double a = A[int64_t(r) * k + c];
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        w[p][q] -= a * wc[q];
                }
            }
        }
    }
}

// Stage 1: w = K(P, S) x(S) for the k pivot points P of a block (forward:
// sigma in X; adjoint: tau in Y) against the rows S of its other box (forward:
// Y; adjoint: X), then the solves; z[rhs][col0 + c].  Lanes: pivot a (A of
// them, a power of two) times source slice q (Q = 64 / A).
template <int NR, int KIND>
__global__ void __launch_bounds__(64)
    k_lu_s1(const LuItem *__restrict__ items, int64_t nitems, const int32_t *__restrict__ piv_row,
            const int32_t *__restrict__ src_off, const int32_t *__restrict__ src_len,
            const int32_t *__restrict__ rank, const int64_t *__restrict__ col0,
            void *const *__restrict__ lu, int adjoint, const double *__restrict__ px,
            const double *__restrict__ py, const double *__restrict__ pz, int kind, double kp,
            const double *__restrict__ xp, int64_t n, int nrhs, int64_t ncols,
            double *__restrict__ z, double *__restrict__ wpart) {
    __shared__ double sx[kLuChunk], sy[kLuChunk], sz[kLuChunk];
    __shared__ double sv[NR][kLuChunk];
    const int64_t w_id = blockIdx.x;
    if (w_id >= nitems)
        return;
    const int lane = threadIdx.x;
    const LuItem it = items[w_id];
    const int b = it.b;
    const int k = rank[b];
    if (k == 0)
        return;
    const int64_t c0 = col0[b];
    const int32_t so = src_off[b], sl = src_len[b];
    const int j0 = it.part < 0 ? 0 : it.part * kLuPart;
    const int j1 = it.part < 0 ? sl : min(sl, j0 + kLuPart);
    int A = 1;
    while (A < k && A < 64)
        A <<= 1;
    const int Q = 64 / A;
    const int al = lane % A, q = lane / A;
    const int npass = (k + 63) >> 6;
    for (int rb = 0; rb < nrhs; rb += NR) {
        double w[kLuSlots][NR];
#pragma unroll
        for (int p = 0; p < kLuSlots; ++p)
#pragma unroll
            for (int c = 0; c < NR; ++c)
                w[p][c] = 0.0;
#pragma unroll
        for (int p = 0; p < kLuSlots; ++p) {
            if (p >= npass)
                break;
            const int a = p * 64 + al;
            const bool aa = a < k;
            const int32_t pr = piv_row[c0 + (aa ? a : 0)];
            const double xi = px[pr], yi = py[pr], zi = pz[pr];
            double acc[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = 0.0;
            for (int cb = j0; cb < j1; cb += kLuChunk) {
                const int cn = min(kLuChunk, j1 - cb);
                __syncthreads();  // the previous chunk's readers are done
#pragma unroll
                for (int u = 0; u < kLuChunk / 64; ++u) {
                    const int f = u * 64 + lane;
                    if (f < cn) {
                        const int64_t gj = int64_t(so) + cb + f;
                        sx[f] = px[gj];
                        sy[f] = py[gj];
                        sz[f] = pz[gj];
#pragma unroll
                        for (int c = 0; c < NR; ++c)
                            sv[c][f] = (rb + c < nrhs) ? xp[(rb + c) * n + gj] : 0.0;
                    }
                }
                __syncthreads();
                if (aa)
                    for (int j = q; j < cn; j += Q) {
                        const double f = entry<KIND>(kind, kp, xi - sx[j], yi - sy[j], zi - sz[j]);
#pragma unroll
                        for (int c = 0; c < NR; ++c)
                            acc[c] += f * sv[c][j];
                    }
            }
            for (int off = A; off < 64; off <<= 1)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    acc[c] += __shfl_xor(acc[c], off, 64);
#pragma unroll
            for (int c = 0; c < NR; ++c)
                w[p][c] = acc[c];
        }
        if (it.part >= 0) {
            // one part of a long source side: partial sums, solved later
            if (q == 0)
                for (int p = 0; p < npass; ++p) {
                    const int a = p * 64 + al;
                    if (a < k)
#pragma unroll
                        for (int c = 0; c < NR; ++c)
                            if (rb + c < nrhs)
                                wpart[(it.wo * nrhs) + int64_t(rb + c) * k + a] = w[p][c];
                }
            continue;
        }
        lu_solve<NR>(static_cast<const double *>(lu[b]), k, adjoint != 0, w);
#pragma unroll
        for (int p = 0; p < kLuSlots; ++p) {
            const int a = p * 64 + lane;
            if (p < npass && a < k && lane < A)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (rb + c < nrhs)
                        z[int64_t(rb + c) * ncols + c0 + a] = w[p][c];
        }
    }
}

// Blocks whose source side was split: the parts' partial sums in part order,
// then the solves.
template <int NR>
__global__ void __launch_bounds__(64)
    k_lu_solve(const LuSplit *__restrict__ items, int64_t nitems, const int32_t *__restrict__ rank,
               const int64_t *__restrict__ col0, void *const *__restrict__ lu, int adjoint,
               int nrhs, int64_t ncols, const double *__restrict__ wpart, double *__restrict__ z) {
    const int64_t w_id = blockIdx.x;
    if (w_id >= nitems)
        return;
    const int lane = threadIdx.x;
    const LuSplit it = items[w_id];
    const int k = rank[it.b];
    if (k == 0)
        return;
    const int64_t c0 = col0[it.b];
    const int npass = (k + 63) >> 6;
    for (int rb = 0; rb < nrhs; rb += NR) {
        double w[kLuSlots][NR];
#pragma unroll
        for (int p = 0; p < kLuSlots; ++p)
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                w[p][c] = 0.0;
                const int a = p * 64 + lane;
                if (p < npass && a < k && rb + c < nrhs)
                    for (int pp = 0; pp < it.np; ++pp)
                        w[p][c] += wpart[(it.wo + int64_t(pp) * k) * nrhs + int64_t(rb + c) * k + a];
            }
        lu_solve<NR>(static_cast<const double *>(lu[it.b]), k, adjoint != 0, w);
#pragma unroll
        for (int p = 0; p < kLuSlots; ++p) {
            const int a = p * 64 + lane;
            if (p < npass && a < k)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (rb + c < nrhs)
                        z[int64_t(rb + c) * ncols + c0 + a] = w[p][c];
        }
    }
}

struct LuS2Tab {
    int64_t box_base[kMaxLevels + 1];
    int L;
};

// Stage 2: one wave per leaf t.  Forward: the columns of the blocks whose
// target contains t (at level l: blocks tgt_begin[g] .. tgt_begin[g + 1] of
// its ancestor g, columns col0 of those) with the tau pivot points; adjoint:
// the blocks whose source contains t, in source-grouped order (positions
// adj_col0 over src_blk, column adj_col[pos]) with the sigma pivot points.
// Lanes: row i (R of them) times column slice q (Q = 64 / R).
template <int NR, int KIND>
__global__ void __launch_bounds__(64)
    k_lu_s2(LuS2Tab tab, const int32_t *__restrict__ leaf_off, const int64_t *__restrict__ grp_begin,
            const int64_t *__restrict__ pos0, const int32_t *__restrict__ pos_col,
            const int32_t *__restrict__ vrow, const double *__restrict__ px,
            const double *__restrict__ py, const double *__restrict__ pz, int kind, double kp,
            const double *__restrict__ z, int64_t ncols, const double *__restrict__ yn, int64_t n,
            int nrhs, const int32_t *__restrict__ perm, void *__restrict__ y, int64_t ldy,
            int io_f32) {
    __shared__ double sx[kLuChunk], sy[kLuChunk], sz[kLuChunk];
    __shared__ double sv[NR][kLuChunk];
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x;
    const int L = tab.L;
    const int32_t t0 = leaf_off[t];
    const int m = leaf_off[t + 1] - t0;
    if (m == 0)
        return;
    int R = 1;
    while (R < m && R < 64)
        R <<= 1;
    const int Q = 64 / R;
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
                acc[c] = (ai && q == 0 && rb + c < nrhs) ? yn[(rb + c) * n + gi] : 0.0;
            for (int l = 1; l <= L; ++l) {
                const int64_t g = tab.box_base[l] + (t >> (3 * (L - l)));
                const int64_t e0 = pos0[grp_begin[g]], e1 = pos0[grp_begin[g + 1]];
                for (int64_t cb = e0; cb < e1; cb += kLuChunk) {
                    const int cn = int(min<int64_t>(kLuChunk, e1 - cb));
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < kLuChunk / 64; ++u) {
                        const int f = u * 64 + lane;
                        if (f < cn) {
                            const int64_t col = pos_col ? int64_t(pos_col[cb + f]) : cb + f;
                            const int32_t vr = vrow[col];
                            sx[f] = px[vr];
                            sy[f] = py[vr];
                            sz[f] = pz[vr];
#pragma unroll
                            for (int c = 0; c < NR; ++c)
                                sv[c][f] = (rb + c < nrhs) ? z[int64_t(rb + c) * ncols + col] : 0.0;
                        }
                    }
                    __syncthreads();
                    if (ai)
                        for (int j = q; j < cn; j += Q) {
                            const double f = entry<KIND>(kind, kp, xi - sx[j], yi - sy[j], zi - sz[j]);
#pragma unroll
                            for (int c = 0; c < NR; ++c)
                                acc[c] += f * sv[c][j];
                        }
                }
            }
            for (int off = R; off < 64; off <<= 1)
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    acc[c] += __shfl_xor(acc[c], off, 64);
            if (ai && q == 0) {
                const int64_t dst = perm[gi];
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (rb + c < nrhs) {
                        if (io_f32)
                            static_cast<float *>(y)[(rb + c) * ldy + dst] = float(acc[c]);
                        else
                            static_cast<double *>(y)[(rb + c) * ldy + dst] = acc[c];
                    }
            }
        }
    }
}

__global__ void k_lu_gather(const void *__restrict__ x, int io_f32, int64_t ldx, int64_t n,
                            int nrhs, const int32_t *__restrict__ perm, double *__restrict__ xp) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n)
        dev::gather_row(x, io_f32, ldx, n, nrhs, perm, xp, p);
}

// ---- build ----------------------------------------------------------------

// packed LU of each block of a finished ACA batch (see the file comment)
__global__ void __launch_bounds__(256)
    k_pack_lu(int64_t q0, int64_t q1, const int32_t *__restrict__ list,
              const int32_t *__restrict__ m, const int32_t *__restrict__ n,
              const int32_t *__restrict__ rank, int max_rank, int kws,
              const double *__restrict__ ws, const int64_t *__restrict__ ws_off, int64_t ws_base,
              const int64_t *__restrict__ off, double *__restrict__ chunk,
              const int32_t *__restrict__ piv, const int64_t *__restrict__ pivoff, void **lu) {
    const int64_t q = q0 + ((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= q1)
        return;
    const int64_t b = list[q];
    const int mb = m[b], nb = n[b], k = rank[b];
    int kcap = mb < nb ? mb : nb;
    if (max_rank > 0 && max_rank < kcap)
        kcap = max_rank;
    kcap = min(kcap, kws);
    const double *U = ws + (ws_off[q] - ws_base);
    const double *V = U + int64_t(mb) * kcap;
    const int32_t *pv = piv + pivoff[b];
    double *d = chunk + off[q - q0];
    for (int64_t e = lane; e < int64_t(k) * k; e += 64) {
        const int c = int(e / k), a = int(e - int64_t(c) * k);  // row a, column c
        d[e] = a >= c ? U[int64_t(c) * mb + pv[2 * a]]        // L[a][c] = u_c[sigma_a]
                      : V[int64_t(a) * nb + pv[2 * c + 1]];   // R[a][c] = v_a[tau_c]
    }
    if (lane == 0)
        lu[b] = d;
}

__global__ void k_lu_sizes(int64_t q0, int64_t q1, const int32_t *__restrict__ list,
                           const int32_t *__restrict__ rank, int64_t *__restrict__ kk) {
    const int64_t q = q0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= q1)
        return;
    const int64_t k = rank[list[q]];
    kk[q - q0] = k * k;
}

// sorted rows of both pivot points of every factor column
__global__ void k_lu_pivot_rows(int64_t nfar, const int32_t *__restrict__ toff,
                                const int32_t *__restrict__ soff, const int32_t *__restrict__ rank,
                                const int64_t *__restrict__ col0, const int32_t *__restrict__ piv,
                                const int64_t *__restrict__ pivoff, int32_t *__restrict__ sig_row,
                                int32_t *__restrict__ tau_row) {
    const int64_t b = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (b >= nfar)
        return;
    const int k = rank[b];
    const int32_t *pv = piv + pivoff[b];
    for (int c = lane; c < k; c += 64) {
        sig_row[col0[b] + c] = toff[b] + pv[2 * c];
        tau_row[col0[b] + c] = soff[b] + pv[2 * c + 1];
    }
}

void check_lu_rank(const Plan &P) {
    if (P.stats.rank_max > kLuMaxRank)
        fail(H3D_ENOTIMPL, "the pivot + LU form solves in registers for ranks up to " +
                               std::to_string(kLuMaxRank) + "; this operator reaches rank " +
                               std::to_string(P.stats.rank_max) + " (set max_rank)");
}

}  // namespace

void lu_pack_batch(Plan &P, const int32_t *list, int64_t q0, int64_t q1, int kws, const double *ws,
                   const int64_t *ws_off, int64_t ws_base, int64_t *scan_buf, hipStream_t s) {
    const int64_t nb = q1 - q0;
    k_lu_sizes<<<grid_for(nb, 256), 256, 0, s>>>(q0, q1, list, P.blk_rank, scan_buf);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipMemsetAsync(scan_buf + nb, 0, sizeof(int64_t), s));
    const int64_t tot = scan_exclusive_i64(P, scan_buf, scan_buf, nb + 1, s);
    if (tot <= 0)
        return;
    double *chunk = P.mem.alloc_n<double>(tot);
    P.chunks.push_back(chunk);
    k_pack_lu<<<grid_for(nb * 64, 256), 256, 0, s>>>(q0, q1, list, P.blk_m, P.blk_n, P.blk_rank,
                                                     P.cfg.max_rank, kws, ws, ws_off, ws_base,
                                                     scan_buf, chunk, P.blk_piv, P.blk_pivoff,
                                                     P.blk_lu);
    H3D_LAUNCH_CHECK();
}

void lu_finish(Plan &P, hipStream_t s) {
    check_lu_rank(P);
    const int64_t nf = P.nfar, nc = std::max<int64_t>(P.ncols, 1);
    P.lu_sig_row = P.mem.alloc_n<int32_t>(nc);
    P.lu_tau_row = P.mem.alloc_n<int32_t>(nc);
    if (nf > 0) {
        k_lu_pivot_rows<<<grid_for(nf * 64, 256), 256, 0, s>>>(nf, P.blk_toff, P.blk_soff,
                                                                P.blk_rank, P.blk_col0, P.blk_piv,
                                                                P.blk_pivoff, P.lu_sig_row,
                                                                P.lu_tau_row);
        H3D_LAUNCH_CHECK();
    }
    // host copies of the block table for the work items
    std::vector<int32_t> rk(static_cast<size_t>(nf)), bm(static_cast<size_t>(nf)), bn(static_cast<size_t>(nf));
    std::vector<int64_t> c0(static_cast<size_t>(nf) + 1), sb(static_cast<size_t>(nf));
    to_host(rk.data(), P.blk_rank, nf, s);
    to_host(bm.data(), P.blk_m, nf, s);
    to_host(bn.data(), P.blk_n, nf, s);
    to_host(c0.data(), P.blk_col0, nf + 1, s);
    to_host(sb.data(), P.src_blk, nf, s);
    // stored bytes: the LU factors, two pivot rows and one adjoint position per
    // column, one adjoint offset per block
    int64_t sq = 0, bytes = 0;
    for (int l = 1; l <= P.L; ++l) {
        int64_t lb = 0;
        for (int64_t b = P.lvl_blk[l]; b < P.lvl_blk[l + 1]; ++b) {
            const int64_t k = rk[size_t(b)];
            sq += k * k;
            lb += k * k * 8 + k * 12 + 8;
        }
        P.stats.factor_bytes_per_level[l] = lb;
        bytes += lb;
    }
    P.lu_sq = sq;
    P.stats.factor_bytes = bytes;
    // adjoint column order: blocks grouped by source box (src_blk), each
    // block's columns in order; adj_col0 over the positions of src_blk
    std::vector<int64_t> adj0(size_t(nf) + 1);
    std::vector<int32_t> adjc(static_cast<size_t>(nc));
    int64_t pos = 0;
    for (int64_t q = 0; q < nf; ++q) {
        adj0[size_t(q)] = pos;
        const int64_t b = sb[size_t(q)];
        for (int c = 0; c < rk[size_t(b)]; ++c)
            adjc[size_t(pos++)] = int32_t(c0[size_t(b)] + c);
    }
    adj0[size_t(nf)] = pos;
    P.lu_adj_col0 = P.mem.alloc_n<int64_t>(nf + 1);
    P.lu_adj_col = P.mem.alloc_n<int32_t>(nc);
    H3D_HIP(hipMemcpyAsync(P.lu_adj_col0, adj0.data(), sizeof(int64_t) * (nf + 1),
                           hipMemcpyHostToDevice, s));
    H3D_HIP(hipMemcpyAsync(P.lu_adj_col, adjc.data(), sizeof(int32_t) * size_t(nc),
                           hipMemcpyHostToDevice, s));
    // stage-1 work items of both directions: a block whose source side
    // (forward: n, adjoint: m) exceeds kLuPart rows is split into parts
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<LuItem> items;
        std::vector<LuSplit> splits;
        items.reserve(size_t(nf));
        int64_t wo = 0;
        for (int64_t b = 0; b < nf; ++b) {
            if (rk[size_t(b)] == 0)
                continue;
            const int len = dir == 0 ? bn[size_t(b)] : bm[size_t(b)];
            if (len <= kLuPart) {
                items.push_back(LuItem{int32_t(b), -1, 0});
                continue;
            }
            const int np = (len + kLuPart - 1) / kLuPart;
            splits.push_back(LuSplit{int32_t(b), np, wo});
            for (int p = 0; p < np; ++p) {
                items.push_back(LuItem{int32_t(b), p, wo});
                wo += rk[size_t(b)];
            }
        }
        P.lu_nitems[dir] = int64_t(items.size());
        P.lu_nsplit[dir] = int64_t(splits.size());
        P.lu_wcols = std::max(P.lu_wcols, wo);
        P.lu_items[dir] = P.mem.alloc(sizeof(LuItem) * std::max<size_t>(items.size(), 1));
        P.lu_split[dir] = P.mem.alloc(sizeof(LuSplit) * std::max<size_t>(splits.size(), 1));
        if (!items.empty())
            H3D_HIP(hipMemcpyAsync(P.lu_items[dir], items.data(), sizeof(LuItem) * items.size(),
                                   hipMemcpyHostToDevice, s));
        if (!splits.empty())
            H3D_HIP(hipMemcpyAsync(P.lu_split[dir], splits.data(), sizeof(LuSplit) * splits.size(),
                                   hipMemcpyHostToDevice, s));
    }
    // partial sums of the split blocks, for up to kLuGroup right-hand sides at once
    P.lu_wpart = P.mem.alloc_n<double>(std::max<int64_t>(P.lu_wcols, 1) * kLuGroup);
    H3D_HIP(hipStreamSynchronize(s));
    // the pivots were kept only for this table, unless asked for
    if (!(P.cfg.flags & H3D_FLAG_KEEP_PIVOTS)) {
        P.mem.release(P.blk_piv);
        P.mem.release(P.blk_pivoff);
        P.blk_piv = nullptr;
        P.blk_pivoff = nullptr;
    }
}

// One product in the pivot + LU form for nrhs <= kLuGroup columns; scratch as
// matvec_vector (xp, yn: n nrhs; z: ncols nrhs).
void matvec_lu(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
               int io_dtype, bool adjoint, double *xp, double *yn, double *z, hipStream_t s) {
    const int64_t n = P.n;
    const int io_f32 = io_dtype == H3D_F32;
    const int nr = int(nrhs);
    const int dir = adjoint ? 1 : 0;
    {
        hipEvent_t ev = P.prof.begin(s);
        k_lu_gather<<<grid_for(n, 256), 256, 0, s>>>(x, io_f32, ldx, n, nr, P.perm, xp);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "k_gather", double(n) * (4.0 + (io_f32 ? 4.0 : 8.0) * nr + 8.0 * nr), 0.0);
    }
    launch_near_field(P, nr, xp, yn, s);
    const bool lap = P.cfg.kernel == H3D_LAPLACE;
    // regenerated entries per product: (m + n) k over all blocks; flops per
    // entry: 3 sub, 5 mul/add, sqrt, division (counted 1 each), 2 per rhs
    const double ev_entries = double(P.stats.factor_entries);
    {
        hipEvent_t ev = P.prof.begin(s);
        const int32_t *prow = adjoint ? P.lu_tau_row : P.lu_sig_row;
        const int32_t *soff = adjoint ? P.blk_toff : P.blk_soff;
        const int32_t *slen = adjoint ? P.blk_m : P.blk_n;
        const LuItem *items = static_cast<const LuItem *>(P.lu_items[dir]);
        if (P.lu_nitems[dir] > 0) {
#define H3D_LU1(NR, K)                                                                           \
    k_lu_s1<NR, K><<<int(P.lu_nitems[dir]), 64, 0, s>>>(                                         \
        items, P.lu_nitems[dir], prow, soff, slen, P.blk_rank, P.blk_col0, P.blk_lu, int(adjoint), \
        P.px, P.py, P.pz, P.cfg.kernel, P.cfg.kernel_param, xp, n, nr, P.ncols, z, P.lu_wpart)
            if (nr == 1) {
                if (lap)
                    H3D_LU1(1, H3D_LAPLACE);
                else
                    H3D_LU1(1, -1);
            } else {
                if (lap)
                    H3D_LU1(kLuNR, H3D_LAPLACE);
                else
                    H3D_LU1(kLuNR, -1);
            }
#undef H3D_LU1
            H3D_LAUNCH_CHECK();
        }
        if (P.lu_nsplit[dir] > 0) {
            const LuSplit *sp = static_cast<const LuSplit *>(P.lu_split[dir]);
            if (nr == 1)
                k_lu_solve<1><<<int(P.lu_nsplit[dir]), 64, 0, s>>>(
                    sp, P.lu_nsplit[dir], P.blk_rank, P.blk_col0, P.blk_lu, int(adjoint), nr,
                    P.ncols, P.lu_wpart, z);
            else
                k_lu_solve<kLuNR><<<int(P.lu_nsplit[dir]), 64, 0, s>>>(
                    sp, P.lu_nsplit[dir], P.blk_rank, P.blk_col0, P.blk_lu, int(adjoint), nr,
                    P.ncols, P.lu_wpart, z);
            H3D_LAUNCH_CHECK();
        }
        const double ent = double(adjoint ? P.stats.factor_entries - P.entries_v : P.entries_v);
        P.prof.end(s, ev, "k_lu_s1", double(P.lu_sq) * 8.0 + double(P.ncols) * (4.0 + 8.0 * nr),
                   ent * (10.0 + 2.0 * nr) + double(P.lu_sq) * 2.0 * nr);
    }
    {
        hipEvent_t ev = P.prof.begin(s);
        LuS2Tab tab{};
        for (int l = 0; l <= kMaxLevels; ++l)
            tab.box_base[l] = P.box_base[l];
        tab.L = P.L;
        const int64_t nleaf = pow8(P.L);
        const int64_t *grp = P.tgt_begin;
        const int64_t *pos0 = adjoint ? P.lu_adj_col0 : P.blk_col0;
        const int32_t *pcol = adjoint ? P.lu_adj_col : nullptr;
        const int32_t *vrow = adjoint ? P.lu_sig_row : P.lu_tau_row;
#define H3D_LU2(NR, K)                                                                           \
    k_lu_s2<NR, K><<<int(nleaf), 64, 0, s>>>(tab, P.leaf_off, grp, pos0, pcol, vrow, P.px, P.py,  \
                                             P.pz, P.cfg.kernel, P.cfg.kernel_param, z, P.ncols, \
                                             yn, n, nr, P.perm, y, ldy, io_f32)
        if (nr == 1) {
            if (lap)
                H3D_LU2(1, H3D_LAPLACE);
            else
                H3D_LU2(1, -1);
        } else {
            if (lap)
                H3D_LU2(kLuNR, H3D_LAPLACE);
            else
                H3D_LU2(kLuNR, -1);
        }
#undef H3D_LU2
        H3D_LAUNCH_CHECK();
        const double ent = double(adjoint ? P.entries_v : P.stats.factor_entries - P.entries_v);
        P.prof.end(s, ev, "k_lu_s2", double(n) * (24.0 + 8.0 * nr + (io_f32 ? 4 : 8) * nr) +
                                         double(P.ncols) * (4.0 + 8.0 * nr),
                   ent * (10.0 + 2.0 * nr));
    }
    (void)ev_entries;
}

void export_lu(const Plan &P, double *host_out) {
    const int64_t nf = P.nfar;
    std::vector<int32_t> rk(static_cast<size_t>(nf));
    std::vector<void *> ptr(static_cast<size_t>(nf));
    to_host(rk.data(), P.blk_rank, nf, nullptr);
    to_host(ptr.data(), P.blk_lu, nf, nullptr);
    int64_t off = 0;
    for (int64_t b = 0; b < nf; ++b) {
        const int64_t kk = int64_t(rk[size_t(b)]) * rk[size_t(b)];
        if (kk > 0)
            H3D_HIP(hipMemcpy(host_out + off, ptr[size_t(b)], sizeof(double) * size_t(kk),
                              hipMemcpyDeviceToHost));
        off += kk;
    }
}

}  // namespace h3d
