// Batched adaptive cross approximation in FP64 (Sec. 4.1, eq. (prank);
// Algorithm 1), with the kernel entries evaluated on the fly from the sorted
// coordinates.
//
// Partially pivoted ACA on block K(X,Y) (rows = target box points, columns =
// source box points, both in sorted order):
//   start at row 0; residual row r = K(i,:) - sum_l u_l[i] v_l;
//   pivot column j = argmax |r_j| over unused columns (ties: lowest j);
//   a row whose residual vanishes on every unused column is skipped in favour
//   of the lowest unused row;
//   v_k = r / r_j;  u_k = K(:,j) - sum_l u_l v_l[j];
//   |S_k|_F^2 += 2 sum_l (u_l.u_k)(v_l.v_k) + |u_k|^2 |v_k|^2;
//   stop once |u_k|^2 |v_k|^2 <= tol^2 |S_k|_F^2, or at k = min(m, n) or the
//   rank cap; next row = argmax |u_k[i]| over unused rows (ties: lowest i).
// Every reduction that feeds a decision runs sequentially in index order and
// no product is contracted into an FMA, so the decisions are reproducible
// run to run and independent of the launch shape.
//
// Two shapes: a sub-wave of SW lanes per block for boxes up to 32 SW points
// (lane r owns rows/columns r, r+SW, ... and keeps their "used" flags in two
// 32-bit masks), and a 256-thread workgroup per block for larger boxes (flags
// in the block's workspace).  Factors go to a per-block FP64 workspace
// [U: m x kcap | V: n x kcap | products: kcap | flags: m + n bytes].
#include "h3d_internal.hpp"

#pragma clang fp contract(off)

namespace h3d {

namespace {

struct Geom {
    const double *px, *py, *pz;
    int kind;
    double kp;
};

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

__device__ __forceinline__ double entry(const Geom &g, int64_t gi, int64_t gj) {
    if (gi == gj)
        return 0.0;
    double dx = g.px[gi] - g.px[gj];
    double dy = g.py[gi] - g.py[gj];
    double dz = g.pz[gi] - g.pz[gj];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    return kernel_f(g.kind, g.kp, r);
}

struct BlockTab {
    const int32_t *toff, *m, *soff, *n;
    const int32_t *list;    // block id of each batch position
    const int64_t *ws_off;  // per position; the batch workspace starts at ws_base
    int64_t ws_base;
    int32_t *rank;
    int32_t *piv;           // optional: 2 kcap ints per block at pivoff
    const int64_t *pivoff;
    unsigned int *ncapped;
    int32_t *overflow;      // set when the workspace column cap stopped the block
    int kws;                // workspace column cap of this pass
};

__device__ __forceinline__ int kcap_of(int m, int n, int max_rank) {
    int k = m < n ? m : n;
    if (max_rank > 0 && max_rank < k)
        k = max_rank;
    return k;
}

// Records how a block ended: a stop at the workspace cap below the real cap
// is not a result (the block is run again with more room); a stop at a rank
// cap below min(m, n) is counted.
__device__ __forceinline__ void finish_block(const BlockTab &T, int64_t b, int k, int m, int n,
                                             int kcap_true, bool hit_cap) {
    if (hit_cap && k < kcap_true) {
        T.overflow[b] = 1;
        T.rank[b] = 0;
        return;
    }
    T.overflow[b] = 0;
    T.rank[b] = k;
    if (hit_cap && kcap_true < (m < n ? m : n))
        atomicAdd(T.ncapped, 1u);
}

// (|value|, index, value) argmax with ties to the lowest index
struct Arg {
    double a;
    int j;
    double v;
};

__device__ __forceinline__ Arg arg_better(Arg x, Arg y) {
    if (y.a > x.a || (y.a == x.a && y.j < x.j))
        return y;
    return x;
}

template <int SW> __device__ __forceinline__ Arg arg_reduce(Arg x) {
#pragma unroll
    for (int off = SW / 2; off > 0; off >>= 1) {
        Arg y;
        y.a = __shfl_xor(x.a, off, SW);
        y.j = __shfl_xor(x.j, off, SW);
        y.v = __shfl_xor(x.v, off, SW);
        x = arg_better(x, y);
    }
    return x;
}

template <int SW> __device__ __forceinline__ int min_reduce(int x) {
#pragma unroll
    for (int off = SW / 2; off > 0; off >>= 1)
        x = min(x, __shfl_xor(x, off, SW));
    return x;
}

constexpr int kNone = 0x7fffffff;

// ---------------------------------------------------------------------------
// one sub-wave of SW lanes per block; a workgroup is one wave (64 / SW blocks)
template <int SW>
__global__ void __launch_bounds__(64)
    k_aca_subwave(int64_t q0, int64_t q1, BlockTab T, Geom G, double tol, int max_rank,
                  double *__restrict__ ws) {
    constexpr int NSUB = 64 / SW;
    const int lane = threadIdx.x;
    const int r = lane % SW;
    const int64_t q = q0 + int64_t(blockIdx.x) * NSUB + lane / SW;
    const bool valid = q < q1;
    int64_t b = 0;
    int m = 0, n = 0, kcap = 0, kcap_true = 0;
    int64_t toff = 0, soff = 0;
    double *U = ws, *V = ws, *P = ws;
    if (valid) {
        b = T.list[q];
        m = T.m[b];
        n = T.n[b];
        toff = T.toff[b];
        soff = T.soff[b];
        kcap_true = kcap_of(m, n, max_rank);
        kcap = min(kcap_true, T.kws);
        U = ws + (T.ws_off[q] - T.ws_base);
        V = U + int64_t(m) * kcap;
        P = V + int64_t(n) * kcap;
    }
    const int mn = m < n ? m : n;
    uint32_t used_r = 0, used_c = 0;  // bit q: row/column r + q SW
    int k = 0, i = 0;
    double S2 = 0.0;
    bool done = !valid || kcap == 0;
    bool capped = false;

    while (__any(!done)) {
        bool act = !done;
        // residual of row i into V[:, k]
        Arg best{-1.0, kNone, 0.0};
        if (act) {
            for (int q = 0, j = r; j < n; ++q, j += SW) {
                double v = entry(G, toff + i, soff + j);
                #pragma unroll 4
                for (int l = 0; l < k; ++l)
                    v -= U[int64_t(l) * m + i] * V[int64_t(l) * n + j];
                V[int64_t(k) * n + j] = v;
                if (!((used_c >> q) & 1u)) {
                    double a = fabs(v);
                    if (a > best.a) {
                        best.a = a;
                        best.j = j;
                        best.v = v;
                    }
                }
            }
            if ((i % SW) == r)
                used_r |= 1u << (i / SW);
        }
        best = arg_reduce<SW>(best);
        // a row already reproduced exactly: continue with the lowest unused row
        const bool exhausted = act && !(best.a > 0.0);
        int low = kNone;
        for (int q = 0, ii = r; ii < m; ++q, ii += SW)
            if (!((used_r >> q) & 1u)) {
                low = ii;
                break;
            }
        low = min_reduce<SW>(low);
        if (exhausted) {
            act = false;
            if (low == kNone)
                done = true;
            else
                i = low;
        }
        const int jp = best.j;
        const double piv = best.v;
        if (act) {
            for (int j = r; j < n; j += SW)
                V[int64_t(k) * n + j] = V[int64_t(k) * n + j] / piv;
            if ((jp % SW) == r)
                used_c |= 1u << (jp / SW);
        }
        __syncthreads();  // V[:, k] and all earlier columns visible to every lane
        if (act) {
            for (int ii = r; ii < m; ii += SW) {
                double v = entry(G, toff + ii, soff + jp);
                #pragma unroll 4
                for (int l = 0; l < k; ++l)
                    v -= U[int64_t(l) * m + ii] * V[int64_t(l) * n + jp];
                U[int64_t(k) * m + ii] = v;
            }
            if (T.piv && r == 0) {
                T.piv[T.pivoff[b] + 2 * k] = i;
                T.piv[T.pivoff[b] + 2 * k + 1] = jp;
            }
        }
        __syncthreads();  // U[:, k] visible
        double uu = 0.0, vv = 0.0;
        if (act) {
            // products (u_l . u_k)(v_l . v_k), one lane per l, sums in index order
            for (int l = r; l < k; l += SW) {
                double a = 0.0, c = 0.0;
                #pragma unroll 8
                for (int ii = 0; ii < m; ++ii)
                    a += U[int64_t(l) * m + ii] * U[int64_t(k) * m + ii];
                #pragma unroll 8
                for (int j = 0; j < n; ++j)
                    c += V[int64_t(l) * n + j] * V[int64_t(k) * n + j];
                P[l] = a * c;
            }
            if (r == 0)
                #pragma unroll 8
                for (int ii = 0; ii < m; ++ii)
                    uu += U[int64_t(k) * m + ii] * U[int64_t(k) * m + ii];
            if (r == (SW > 1 ? 1 : 0))
                #pragma unroll 8
                for (int j = 0; j < n; ++j)
                    vv += V[int64_t(k) * n + j] * V[int64_t(k) * n + j];
        }
        __syncthreads();  // products visible
        uu = __shfl(uu, 0, SW);
        vv = __shfl(vv, SW > 1 ? 1 : 0, SW);
        Arg nx{-1.0, kNone, 0.0};
        if (act) {
            double cross = 0.0;
            for (int l = 0; l < k; ++l)
                cross += P[l];
            S2 = S2 + 2.0 * cross + uu * vv;
            k += 1;
            if (uu * vv <= tol * tol * S2 || k == mn) {
                done = true;
            } else if (k == kcap) {
                done = true;
                capped = true;
            }
            for (int q = 0, ii = r; ii < m; ++q, ii += SW)
                if (!((used_r >> q) & 1u)) {
                    double a = fabs(U[int64_t(k - 1) * m + ii]);
                    if (a > nx.a) {
                        nx.a = a;
                        nx.j = ii;
                    }
                }
        }
        nx = arg_reduce<SW>(nx);
        if (act && !done) {
            if (nx.j == kNone)
                done = true;
            else
                i = nx.j;
        }
        __syncthreads();
    }
    if (valid && r == 0)
        finish_block(T, b, k, m, n, kcap_true, capped);
}

// ---------------------------------------------------------------------------
// one 256-thread workgroup per block, for boxes larger than 32 SW points
constexpr int kWG = 256;

__device__ __forceinline__ Arg wg_arg_reduce(Arg x, Arg *sh) {
    // wave level, then across the 4 waves through LDS
    x = arg_reduce<64>(x);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        sh[w] = x;
    __syncthreads();
    Arg r = sh[0];
    for (int q = 1; q < kWG / 64; ++q)
        r = arg_better(r, sh[q]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kWG)
    k_aca_workgroup(int64_t q0, BlockTab T, Geom G, double tol, int max_rank,
                    double *__restrict__ ws) {
    __shared__ Arg sh_arg[kWG / 64];
    __shared__ double sh_uv[2];
    const int tid = threadIdx.x;
    const int64_t q = q0 + blockIdx.x;
    const int64_t b = T.list[q];
    const int m = T.m[b], n = T.n[b];
    const int64_t toff = T.toff[b], soff = T.soff[b];
    const int kcap_true = kcap_of(m, n, max_rank);
    const int kcap = min(kcap_true, T.kws);
    const int mn = m < n ? m : n;
    double *U = ws + (T.ws_off[q] - T.ws_base);
    double *V = U + int64_t(m) * kcap;
    double *P = V + int64_t(n) * kcap;
    unsigned char *used_r = reinterpret_cast<unsigned char *>(P + kcap);
    unsigned char *used_c = used_r + m;
    for (int ii = tid; ii < m; ii += kWG)
        used_r[ii] = 0;
    for (int j = tid; j < n; j += kWG)
        used_c[j] = 0;
    __syncthreads();
    int k = 0, i = 0;
    double S2 = 0.0;
    bool capped = false;
    bool done = kcap == 0;
    while (!done) {
        Arg best{-1.0, kNone, 0.0};
        for (int j = tid; j < n; j += kWG) {
            double v = entry(G, toff + i, soff + j);
            #pragma unroll 4
            for (int l = 0; l < k; ++l)
                v -= U[int64_t(l) * m + i] * V[int64_t(l) * n + j];
            V[int64_t(k) * n + j] = v;
            if (!used_c[j]) {
                double a = fabs(v);
                if (a > best.a) {
                    best.a = a;
                    best.j = j;
                    best.v = v;
                }
            }
        }
        if (tid == 0)
            used_r[i] = 1;
        best = wg_arg_reduce(best, sh_arg);  // includes barriers: used_r[i] visible
        if (!(best.a > 0.0)) {
            // lowest unused row
            Arg low{-1.0, kNone, 0.0};
            for (int ii = tid; ii < m; ii += kWG)
                if (!used_r[ii]) {
                    low = Arg{0.0, ii, 0.0};
                    break;
                }
            low = wg_arg_reduce(low, sh_arg);
            if (low.j == kNone)
                break;
            i = low.j;
            continue;
        }
        const int jp = best.j;
        const double piv = best.v;
        for (int j = tid; j < n; j += kWG)
            V[int64_t(k) * n + j] = V[int64_t(k) * n + j] / piv;
        __syncthreads();
        for (int ii = tid; ii < m; ii += kWG) {
            double v = entry(G, toff + ii, soff + jp);
            #pragma unroll 4
            for (int l = 0; l < k; ++l)
                v -= U[int64_t(l) * m + ii] * V[int64_t(l) * n + jp];
            U[int64_t(k) * m + ii] = v;
        }
        if (tid == 0) {
            used_c[jp] = 1;
            if (T.piv) {
                T.piv[T.pivoff[b] + 2 * k] = i;
                T.piv[T.pivoff[b] + 2 * k + 1] = jp;
            }
        }
        __syncthreads();
        for (int l = tid; l < k; l += kWG) {
            double a = 0.0, c = 0.0;
            #pragma unroll 8
            for (int ii = 0; ii < m; ++ii)
                a += U[int64_t(l) * m + ii] * U[int64_t(k) * m + ii];
            #pragma unroll 8
            for (int j = 0; j < n; ++j)
                c += V[int64_t(l) * n + j] * V[int64_t(k) * n + j];
            P[l] = a * c;
        }
        if (tid == kWG - 1) {
            double uu = 0.0;
            #pragma unroll 8
            for (int ii = 0; ii < m; ++ii)
                uu += U[int64_t(k) * m + ii] * U[int64_t(k) * m + ii];
            sh_uv[0] = uu;
        }
        if (tid == kWG - 2) {
            double vv = 0.0;
            #pragma unroll 8
            for (int j = 0; j < n; ++j)
                vv += V[int64_t(k) * n + j] * V[int64_t(k) * n + j];
            sh_uv[1] = vv;
        }
        __syncthreads();
        const double uu = sh_uv[0], vv = sh_uv[1];
        double cross = 0.0;
        for (int l = 0; l < k; ++l)
            cross += P[l];
        S2 = S2 + 2.0 * cross + uu * vv;
        k += 1;
        if (uu * vv <= tol * tol * S2 || k == mn)
            break;
        if (k == kcap) {
            capped = true;
            break;
        }
        Arg nx{-1.0, kNone, 0.0};
        for (int ii = tid; ii < m; ii += kWG)
            if (!used_r[ii]) {
                double a = fabs(U[int64_t(k - 1) * m + ii]);
                if (a > nx.a) {
                    nx.a = a;
                    nx.j = ii;
                }
            }
        nx = wg_arg_reduce(nx, sh_arg);
        if (nx.j == kNone)
            break;
        i = nx.j;
    }
    if (tid == 0)
        finish_block(T, b, k, m, n, kcap_true, capped);
}

// workspace doubles of each listed block for a pass with column cap kws
__global__ void k_ws_size(int64_t cnt, const int32_t *__restrict__ list,
                          const int32_t *__restrict__ m, const int32_t *__restrict__ n,
                          int max_rank, int kws, int64_t *__restrict__ ws) {
    int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= cnt)
        return;
    const int64_t b = list[q];
    int64_t kc = min(kcap_of(m[b], n[b], max_rank), kws);
    ws[q] = (int64_t(m[b]) + n[b]) * kc + kc + (int64_t(m[b]) + n[b] + 7) / 8 + 1;
}

// pivot slots (2 per possible rank) of every block
__global__ void k_piv_size(int64_t nfar, const int32_t *__restrict__ m, const int32_t *__restrict__ n,
                           int max_rank, int64_t *__restrict__ kc) {
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b < nfar)
        kc[b] = 2 * int64_t(kcap_of(m[b], n[b], max_rank));
}

}  // namespace

// Runs ACA over positions [q0, q1) of the batch list (one level) into the
// workspace ws, whose per-position offsets relative to ws_base are ws_off.
void aca_level_batch(Plan &P, int level, const int32_t *list, int64_t q0, int64_t q1, double *ws,
                     const int64_t *ws_off, int64_t ws_base, int kws, int32_t *overflow,
                     unsigned int *ncapped, hipStream_t s) {
    if (q1 <= q0)
        return;
    Geom G{P.px, P.py, P.pz, P.cfg.kernel, P.cfg.kernel_param};
    BlockTab T{P.blk_toff, P.blk_m, P.blk_soff, P.blk_n, list, ws_off, ws_base, P.blk_rank,
               P.blk_piv, P.blk_pivoff, ncapped, overflow, kws};
    const int mx = P.max_box[level];
    const int64_t nb = q1 - q0;
    const double tol = P.cfg.tol;
    const int mr = P.cfg.max_rank;
    if (mx <= 32 * 4) {
        // small boxes: pack several blocks into one wave
        int sw = 4;
        while (sw < 64 && sw < P.mean_box[level])
            sw *= 2;
        while (32 * sw < mx)
            sw *= 2;
        switch (sw) {
        case 4:
            k_aca_subwave<4><<<grid_for(nb, 16), 64, 0, s>>>(q0, q1, T, G, tol, mr, ws);
            break;
        case 8:
            k_aca_subwave<8><<<grid_for(nb, 8), 64, 0, s>>>(q0, q1, T, G, tol, mr, ws);
            break;
        case 16:
            k_aca_subwave<16><<<grid_for(nb, 4), 64, 0, s>>>(q0, q1, T, G, tol, mr, ws);
            break;
        case 32:
            k_aca_subwave<32><<<grid_for(nb, 2), 64, 0, s>>>(q0, q1, T, G, tol, mr, ws);
            break;
        default:
            k_aca_subwave<64><<<grid_for(nb, 1), 64, 0, s>>>(q0, q1, T, G, tol, mr, ws);
            break;
        }
    } else if (mx <= 32 * 64) {
        k_aca_subwave<64><<<grid_for(nb, 1), 64, 0, s>>>(q0, q1, T, G, tol, mr, ws);
    } else {
        k_aca_workgroup<<<int(nb), kWG, 0, s>>>(q0, T, G, tol, mr, ws);
    }
    H3D_LAUNCH_CHECK();
}

void aca_workspace_sizes(Plan &P, const int32_t *list, int64_t cnt, int kws, int64_t *ws,
                         hipStream_t s) {
    if (cnt <= 0)
        return;
    k_ws_size<<<grid_for(cnt, 256), 256, 0, s>>>(cnt, list, P.blk_m, P.blk_n, P.cfg.max_rank, kws,
                                                 ws);
    H3D_LAUNCH_CHECK();
}

void aca_pivot_sizes(Plan &P, int64_t *kc2, hipStream_t s) {
    if (P.nfar <= 0)
        return;
    k_piv_size<<<grid_for(P.nfar, 256), 256, 0, s>>>(P.nfar, P.blk_m, P.blk_n, P.cfg.max_rank, kc2);
    H3D_LAUNCH_CHECK();
}

}  // namespace h3d
