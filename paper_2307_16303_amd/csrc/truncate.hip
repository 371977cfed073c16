// Rank truncation of the ACA factors in FP64 (optional, H3D_FLAG_TRUNCATE).
//
// ACA (Sec. 4.1, eq. (prank)) stops on an estimate, so its rank k is often
// larger than the numerical rank of U V^T at the same tolerance (the
// notation section's epsilon-rank).  Recompression, as the references of
// Sec. 4.1 describe it, brings U V^T to its optimal rank:
//
//   U = Q_U R_U, V = Q_V R_V          (Householder QR, FP64)
//   R_U R_V^T = W S Z^T               (SVD of the k x k core, one-sided Jacobi)
//   r = the smallest rank with ||(s_{r+1}, ..., s_k)||_2 <= tol ||s||_2
//   U' = Q_U W_r S_r^(1/2),  V' = Q_V Z_r S_r^(1/2)
//
// so U' V'^T is the best rank-r approximation of U V^T and differs from it
// by at most tol ||U V^T||_F.
//
// One wave per block, on the block's FP64 ACA workspace (U: m x k, V: n x k,
// column-major) right after ACA and before packing.  Row i of every m x .,
// n x . or k x . array belongs to lane i mod 64 throughout, so each element is
// read and written by one lane only and lanes exchange values through
// shuffles and a wave-private LDS area; every sum is a fixed-order wave
// reduction, so the result is deterministic.  Blocks of rank < 2 or > 256,
// boxes of more than 4096 points and blocks that ACA has to run again are
// left as they are.
#include "h3d_internal.hpp"

namespace h3d {

namespace {

constexpr int kTruncMaxRank = 256;
// one wave streams a factor k^2/2 times during its QR, which for boxes of
// many thousands of rows is a long latency-bound walk over HBM: such blocks
// (levels 1-2 of large clouds) keep their ACA factors
constexpr int kTruncMaxRows = 4096;
constexpr int kJacobiSweeps = 15;
constexpr int kTruncWaves = 4;  // waves (blocks) per workgroup

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// orders LDS accesses of the wave (LDS operations of one wave complete in
// order; this keeps the compiler from moving them across)
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Householder QR in place: A (rows x k, leading dimension ld) becomes R
// (upper triangle) and the reflectors v_j (below the diagonal, v_j[j] = 1
// implied); tau[j] in LDS.
__device__ void house_qr(double *A, int rows, int64_t ld, int k, double *tau, int lane) {
    for (int j = 0; j < k; ++j) {
        double *a = A + int64_t(j) * ld;
        double s = 0.0;
        for (int i = j + 1 + lane; i < rows; i += 64)
            s += a[i] * a[i];
        s = wsum(s);
        const int oj = j & 63;
        const double alpha = __shfl(lane == oj ? a[j] : 0.0, oj, 64);
        double t = 0.0, scale = 0.0, beta = alpha;
        if (s > 0.0) {
            const double nrm = sqrt(alpha * alpha + s);
            beta = alpha >= 0.0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        for (int i = j + 1 + lane; i < rows; i += 64)
            a[i] *= scale;  // v_j below the diagonal (zero when t = 0)
        if (lane == oj)
            a[j] = beta;
        if (lane == 0)
            tau[j] = t;
        // apply H_j = I - t v v^T to the remaining columns
        if (t != 0.0)
            for (int c = j + 1; c < k; ++c) {
                double *b = A + int64_t(c) * ld;
                double w = 0.0;
                for (int i = j + 1 + lane; i < rows; i += 64)
                    w += a[i] * b[i];
                w = wsum(w) + __shfl(lane == oj ? b[j] : 0.0, oj, 64);
                const double tw = t * w;
                if (lane == oj)
                    b[j] -= tw;
                for (int i = j + 1 + lane; i < rows; i += 64)
                    b[i] -= tw * a[i];
            }
    }
    wave_fence();
}

// X (rows x r, leading dimension ldx) <- Q X, Q = H_0 H_1 ... H_{k-1} from house_qr
__device__ void apply_q(const double *A, int rows, int64_t ld, int k, const double *tau, double *X,
                        int64_t ldx, int r, int lane) {
    for (int j = k - 1; j >= 0; --j) {
        const double t = tau[j];
        if (t == 0.0)
            continue;
        const double *a = A + int64_t(j) * ld;
        const int oj = j & 63;
        for (int c = 0; c < r; ++c) {
            double *x = X + int64_t(c) * ldx;
            double w = 0.0;
            for (int i = j + 1 + lane; i < rows; i += 64)
                w += a[i] * x[i];
            w = wsum(w) + __shfl(lane == oj ? x[j] : 0.0, oj, 64);
            const double tw = t * w;
            if (lane == oj)
                x[j] -= tw;
            for (int i = j + 1 + lane; i < rows; i += 64)
                x[i] -= tw * a[i];
        }
    }
}

__global__ void __launch_bounds__(64 * kTruncWaves)
    k_truncate(int64_t q0, int64_t q1, const int32_t *__restrict__ list,
               const int32_t *__restrict__ m, const int32_t *__restrict__ n, int32_t *rank,
               const int32_t *__restrict__ overflow, int max_rank, int kws, double *ws,
               const int64_t *__restrict__ ws_off, int64_t ws_base, double *tmp,
               const int64_t *__restrict__ tmp_off, double tol) {
    __shared__ double sh_tau[kTruncWaves][2][kTruncMaxRank];
    __shared__ double sh_sig[kTruncWaves][kTruncMaxRank];
    __shared__ int sh_ord[kTruncWaves][kTruncMaxRank];
    __shared__ int sh_r[kTruncWaves];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = q0 + int64_t(blockIdx.x) * kTruncWaves + wv;
    if (q >= q1)
        return;
    const int64_t b = list[q];
    const int k = rank[b];
    const int mb = m[b], nb = n[b];
    if (k < 2 || k > kTruncMaxRank || overflow[b] || mb > kTruncMaxRows || nb > kTruncMaxRows)
        return;
    int kcap = mb < nb ? mb : nb;
    if (max_rank > 0 && max_rank < kcap)
        kcap = max_rank;
    kcap = min(kcap, kws);
    double *U = ws + (ws_off[q] - ws_base);
    double *V = U + int64_t(mb) * kcap;
    // QR of copies: U and V stay the ACA factors unless the rank drops
    double *QU = tmp + tmp_off[q - q0];
    double *QV = QU + int64_t(mb) * k;
    double *C = QV + int64_t(nb) * k;
    double *Z = C + int64_t(k) * k;
    double *tauU = sh_tau[wv][0], *tauV = sh_tau[wv][1];
    double *sig = sh_sig[wv];
    int *ord = sh_ord[wv];
    for (int c = 0; c < k; ++c) {
        for (int i = lane; i < mb; i += 64)
            QU[i + int64_t(c) * mb] = U[i + int64_t(c) * mb];
        for (int i = lane; i < nb; i += 64)
            QV[i + int64_t(c) * nb] = V[i + int64_t(c) * nb];
    }

    house_qr(QU, mb, mb, k, tauU, lane);
    house_qr(QV, nb, nb, k, tauV, lane);

    // core C = R_U R_V^T (k x k), Z = I
    for (int j = 0; j < k; ++j) {
        const int oj = j & 63;
        for (int i = lane; i < k; i += 64) {
            C[i + int64_t(j) * k] = 0.0;
            Z[i + int64_t(j) * k] = i == j ? 1.0 : 0.0;
        }
        for (int l = j; l < k; ++l) {
            const double rv = __shfl(lane == oj ? QV[j + int64_t(l) * nb] : 0.0, oj, 64);
            for (int i = lane; i <= l && i < k; i += 64)
                C[i + int64_t(j) * k] += QU[i + int64_t(l) * mb] * rv;
        }
    }

    // one-sided Jacobi: rotate columns of C (and Z) until they are orthogonal.
    // Row i of C and Z lives with lane i mod 64, at most kTruncMaxRank / 64
    // rows per lane, so a pair of columns is held in registers while rotated.
    // Columns below 1e-15 of the core's Frobenius norm are left alone: they
    // are dropped by any tolerance the build accepts.
    constexpr int RPL = kTruncMaxRank / 64;
    double fro = 0.0;
    for (int c = 0; c < k; ++c)
        for (int i = lane; i < k; i += 64)
            fro += C[i + int64_t(c) * k] * C[i + int64_t(c) * k];
    fro = wsum(fro);
    const double tiny = 1e-30 * fro;
    for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < k - 1; ++p)
            for (int qq = p + 1; qq < k; ++qq) {
                double *cp = C + int64_t(p) * k, *cq = C + int64_t(qq) * k;
                double xp[RPL], xq[RPL];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int i = lane + 64 * t;
                    xp[t] = i < k ? cp[i] : 0.0;
                    xq[t] = i < k ? cq[i] : 0.0;
                    al += xp[t] * xp[t];
                    be += xq[t] * xq[t];
                    ga += xp[t] * xq[t];
                }
                al = wsum(al);
                be = wsum(be);
                ga = wsum(ga);
                if (ga == 0.0 || al <= tiny || be <= tiny)
                    continue;
                const double rel = fabs(ga) / sqrt(al * be);
                off = fmax(off, rel);
                if (rel < 1e-14)
                    continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                double *zp = Z + int64_t(p) * k, *zq = Z + int64_t(qq) * k;
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int i = lane + 64 * t;
                    if (i < k) {
                        cp[i] = cs * xp[t] - sn * xq[t];
                        cq[i] = sn * xp[t] + cs * xq[t];
                        const double u = zp[i], v = zq[i];
                        zp[i] = cs * u - sn * v;
                        zq[i] = sn * u + cs * v;
                    }
                }
            }
        if (off < 1e-14)
            break;
    }

    // singular values, their order (descending, ties by index), kept rank
    for (int c = 0; c < k; ++c) {
        const double *cc = C + int64_t(c) * k;
        double s2 = 0.0;
        for (int i = lane; i < k; i += 64)
            s2 += cc[i] * cc[i];
        s2 = wsum(s2);
        if (lane == 0)
            sig[c] = sqrt(s2);
    }
    wave_fence();
    for (int c = lane; c < k; c += 64) {
        int rk = 0;
        for (int j = 0; j < k; ++j)
            rk += (sig[j] > sig[c] || (sig[j] == sig[c] && j < c)) ? 1 : 0;
        ord[rk] = c;
    }
    wave_fence();
    if (lane == 0) {
        double tot = 0.0;
        for (int t = 0; t < k; ++t)
            tot += sig[ord[t]] * sig[ord[t]];
        const double lim = tol * tol * tot;
        double tail = 0.0;
        int r = k;
        while (r > 1) {
            const double s = sig[ord[r - 1]];
            if (tail + s * s > lim)
                break;
            tail += s * s;
            --r;
        }
        sh_r[wv] = tot > 0.0 ? r : k;
    }
    wave_fence();
    const int r = sh_r[wv];
    if (r >= k)
        return;  // nothing to drop: the ACA factors stay

    // U' = Q_U [W_r S_r^(1/2); 0],  V' = Q_V [Z_r S_r^(1/2); 0], written over
    // the first r columns of U and V
    for (int c = 0; c < r; ++c) {
        const int oc = ord[c];
        const double s = sig[oc];
        const double iu = s > 0.0 ? 1.0 / sqrt(s) : 0.0, sv = sqrt(s);
        for (int i = lane; i < mb; i += 64)
            U[i + int64_t(c) * mb] = i < k ? C[i + int64_t(oc) * k] * iu : 0.0;
        for (int i = lane; i < nb; i += 64)
            V[i + int64_t(c) * nb] = i < k ? Z[i + int64_t(oc) * k] * sv : 0.0;
    }
    apply_q(QU, mb, mb, k, tauU, U, mb, r, lane);
    apply_q(QV, nb, nb, k, tauV, V, nb, r, lane);
    if (lane == 0)
        rank[b] = r;
}

__global__ void k_trunc_sizes(int64_t q0, int64_t q1, const int32_t *__restrict__ list,
                              const int32_t *__restrict__ m, const int32_t *__restrict__ n,
                              const int32_t *__restrict__ rank, int64_t *__restrict__ sz) {
    const int64_t q = q0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= q1)
        return;
    const int64_t b = list[q];
    const int64_t k = rank[b];
    const bool on = k >= 2 && k <= kTruncMaxRank && m[b] <= kTruncMaxRows && n[b] <= kTruncMaxRows;
    sz[q - q0] = on ? (int64_t(m[b]) + n[b]) * k + 2 * k * k : 0;
}

}  // namespace

// Truncates the blocks list[q0..q1) whose ACA factors sit in the workspace.
void truncate_batch(Plan &P, const int32_t *list, int64_t q0, int64_t q1, int kws, double *ws,
                    const int64_t *ws_off, int64_t ws_base, const int32_t *overflow,
                    hipStream_t s) {
    const int64_t nb = q1 - q0;
    if (nb <= 0)
        return;
    int64_t *off = P.mem.alloc_n<int64_t>(nb + 1);
    k_trunc_sizes<<<grid_for(nb, 256), 256, 0, s>>>(q0, q1, list, P.blk_m, P.blk_n, P.blk_rank, off);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipMemsetAsync(off + nb, 0, sizeof(int64_t), s));
    const int64_t tot = scan_exclusive_i64(P, off, off, nb + 1, s);
    if (tot > 0) {
        double *tmp = P.mem.alloc_n<double>(tot);
        k_truncate<<<int(ceil_div(nb, kTruncWaves)), 64 * kTruncWaves, 0, s>>>(
            q0, q1, list, P.blk_m, P.blk_n, P.blk_rank, overflow, P.cfg.max_rank, kws, ws, ws_off,
            ws_base, tmp, off, P.cfg.tol);
        H3D_LAUNCH_CHECK();
        H3D_HIP(hipStreamSynchronize(s));
        P.mem.release(tmp);
    }
    P.mem.release(off);
}

}  // namespace h3d
