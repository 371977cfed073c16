// The HODLR3D product inside an iterative solver (Sec. 5.2): restarted GMRES
// for (diag I + scale K~) x = f, the discrete second-kind integral equation of
// eqs. (IE) and (ILDiscrete) with K~ the plan's operator, and the exact dense
// product y = K x that gives a right-hand side "exact up to roundoff".
//
// GMRES(m) (Saad and Schultz): the Krylov basis lives on the device (n x
// (m + 1), caller point order); each iteration is one HODLR3D product plus
// classical Gram-Schmidt with one reorthogonalisation (CGS2: the projections
// on all earlier basis vectors in one pass over the rows, twice), so a step
// needs one small device-to-host copy (the Hessenberg column and the norm).
// Every dot product is reduced in a fixed order (per-workgroup partial sums,
// then one workgroup over them): solves are bitwise reproducible.  The Givens
// rotations and the small least-squares solve run on the host; every cycle
// ends with the true residual f - A x.
#include <cmath>
#include <vector>

#include "product_items.hpp"

namespace h3d {

namespace {

constexpr int kDotBlock = 256;
constexpr int kDotGrid = 512;   // partial sums per dot product

// w = a v + b w
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ v, double b,
                        double *__restrict__ w) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        w[i] = a * v[i] + b * w[i];
}

// r = f - (a x + b y)
__global__ void k_residual(int64_t n, const double *__restrict__ f, double a,
                           const double *__restrict__ x, double b, const double *__restrict__ y,
                           double *__restrict__ r) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        r[i] = f[i] - (a * x[i] + b * y[i]);
}

// part[g][c] = sum over rows i of workgroup g's stride of V[c][i] w[i], c < nv
__global__ void __launch_bounds__(kDotBlock)
    k_dots_part(int64_t n, const double *__restrict__ V, int64_t ldv, int nv,
                const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double red[kDotBlock];
    for (int c = 0; c < nv; ++c) {
        double acc = 0.0;
        for (int64_t i = int64_t(blockIdx.x) * kDotBlock + threadIdx.x; i < n;
             i += int64_t(gridDim.x) * kDotBlock)
            acc += V[c * ldv + i] * w[i];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int off = kDotBlock / 2; off > 0; off >>= 1) {
            if (int(threadIdx.x) < off)
                red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            part[int64_t(blockIdx.x) * nv + c] = red[0];
        __syncthreads();
    }
}

// out[c] (+)= sum over g of part[g][c], g ascending
__global__ void k_dots_sum(int ng, int nv, const double *__restrict__ part, double *__restrict__ out,
                           int accumulate) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nv)
        return;
    double s = 0.0;
    for (int g = 0; g < ng; ++g)
        s += part[int64_t(g) * nv + c];
    out[c] = accumulate ? out[c] + s : s;
}

// w[i] -= sum_c V[c][i] h[c]  (or x[i] += ..., sign = +1)
__global__ void k_combine(int64_t n, const double *__restrict__ V, int64_t ldv, int nv,
                          const double *__restrict__ h, double sign, double *__restrict__ w) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double s = 0.0;
    for (int c = 0; c < nv; ++c)
        s += V[c * ldv + i] * h[c];
    w[i] += sign * s;
}

__global__ void k_scale_copy(int64_t n, double a, const double *__restrict__ w,
                             double *__restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        v[i] = a * w[i];
}

// y_i = sum_{j != i} f(|p_i - p_j|) x_j over every point (caller order); one
// thread per target row, sources staged through LDS
constexpr int kDenseTile = 256;
template <int KIND>
__global__ void __launch_bounds__(kDenseTile)
    k_dense(const double *__restrict__ pts, int64_t n, int kind, double kp,
            const double *__restrict__ x, double *__restrict__ y) {
    __shared__ double sx[kDenseTile], sy[kDenseTile], sz[kDenseTile], sv[kDenseTile];
    const int64_t i = int64_t(blockIdx.x) * kDenseTile + threadIdx.x;
    const bool ai = i < n;
    const int64_t ic = ai ? i : 0;
    const double xi = pts[3 * ic], yi = pts[3 * ic + 1], zi = pts[3 * ic + 2];
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kDenseTile) {
        const int64_t j = j0 + threadIdx.x;
        __syncthreads();
        if (j < n) {
            sx[threadIdx.x] = pts[3 * j];
            sy[threadIdx.x] = pts[3 * j + 1];
            sz[threadIdx.x] = pts[3 * j + 2];
            sv[threadIdx.x] = x[j];
        }
        __syncthreads();
        const int cnt = int(min<int64_t>(kDenseTile, n - j0));
        if (ai)
            for (int q = 0; q < cnt; ++q) {
                if (j0 + q == i)
                    continue;
                const double dx = xi - sx[q], dy = yi - sy[q], dz = zi - sz[q];
                acc += dev::kernel_f(KIND >= 0 ? KIND : kind, kp, sqrt(dx * dx + dy * dy + dz * dz)) *
                       sv[q];
            }
    }
    if (ai)
        y[i] = acc;
}

}  // namespace

void dense_matvec(const double *pts, int64_t n, int kind, double kp, const double *x, double *y,
                  hipStream_t s) {
    const int g = grid_for(n, kDenseTile);
    if (kind == H3D_LAPLACE)
        k_dense<H3D_LAPLACE><<<g, kDenseTile, 0, s>>>(pts, n, kind, kp, x, y);
    else
        k_dense<-1><<<g, kDenseTile, 0, s>>>(pts, n, kind, kp, x, y);
    H3D_LAUNCH_CHECK();
}

SolveResult solve_gmres(Plan &P, double diag, double scale, const double *f, double *x,
                        double rtol, int restart, int max_iter, hipStream_t s) {
    const int64_t n = P.n;
    const int m = restart;
    const int tb = 256, gn = grid_for(n, tb);
    // device work space, returned to the plan's allocator at the end
    double *V = P.mem.alloc_n<double>(n * (m + 1));
    double *w = P.mem.alloc_n<double>(n);
    double *part = P.mem.alloc_n<double>(int64_t(kDotGrid) * (m + 2));
    double *hd = P.mem.alloc_n<double>(m + 2);
    SolveResult res{};
    auto cleanup = [&] {
        (void)hipStreamSynchronize(s);
        P.mem.release(V);
        P.mem.release(w);
        P.mem.release(part);
        P.mem.release(hd);
    };
    try {
        // w = A v = diag v + scale K~ v
        auto apply = [&](const double *v, double *out) {
            matvec_run(P, v, out, 1, n, n, H3D_F64, false, s);
            k_axpby<<<gn, tb, 0, s>>>(n, diag, v, scale, out);
            H3D_LAUNCH_CHECK();
        };
        // hd[0..nv) (+)= V[0..nv)^T u
        auto dots = [&](const double *Vb, int nv, const double *u, int accumulate) {
            k_dots_part<<<kDotGrid, kDotBlock, 0, s>>>(n, Vb, n, nv, u, part);
            H3D_LAUNCH_CHECK();
            k_dots_sum<<<grid_for(nv, 64), 64, 0, s>>>(kDotGrid, nv, part, hd, accumulate);
            H3D_LAUNCH_CHECK();
        };
        auto norm = [&](const double *u) {
            dots(u, 1, u, 0);
            double v = 0.0;
            to_host(&v, hd, 1, s);
            return std::sqrt(v);
        };
        double fn = norm(f);
        if (fn == 0.0) {
            H3D_HIP(hipMemsetAsync(x, 0, sizeof(double) * size_t(n), s));
            res.converged = 1;
            cleanup();
            return res;
        }
        const size_t ms = static_cast<size_t>(m);
        std::vector<double> H((ms + 1) * ms), cs(ms), sn(ms), g(ms + 1), hc(ms + 2), y(ms);
        int it = 0;
        for (;;) {
            // r = f - A x into basis vector 0
            apply(x, w);
            k_residual<<<gn, tb, 0, s>>>(n, f, 0.0, x, 1.0, w, V);
            H3D_LAUNCH_CHECK();
            const double beta = norm(V);
            res.rel_residual = beta / fn;
            if (beta / fn < rtol || it >= max_iter) {
                res.converged = beta / fn < rtol;
                break;
            }
            k_scale_copy<<<gn, tb, 0, s>>>(n, 1.0 / beta, V, V);
            H3D_LAUNCH_CHECK();
            std::fill(H.begin(), H.end(), 0.0);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int jj = 0;
            for (int j = 0; j < m; ++j) {
                double *vj = V + int64_t(j) * n;
                apply(vj, w);
                ++it;
                // CGS2: h = V^T w; w -= V h; twice
                dots(V, j + 1, w, 0);
                k_combine<<<gn, tb, 0, s>>>(n, V, n, j + 1, hd, -1.0, w);
                H3D_LAUNCH_CHECK();
                std::vector<double> h1(size_t(j) + 1);
                to_host(h1.data(), hd, j + 1, s);
                dots(V, j + 1, w, 0);
                k_combine<<<gn, tb, 0, s>>>(n, V, n, j + 1, hd, -1.0, w);
                H3D_LAUNCH_CHECK();
                to_host(hc.data(), hd, j + 1, s);
                for (int i = 0; i <= j; ++i)
                    H[size_t(i) * m + j] = h1[size_t(i)] + hc[size_t(i)];
                const double hn = norm(w);
                H[size_t(j + 1) * m + j] = hn;
                if (hn > 0.0) {
                    k_scale_copy<<<gn, tb, 0, s>>>(n, 1.0 / hn, w, V + int64_t(j + 1) * n);
                    H3D_LAUNCH_CHECK();
                }
                for (int i = 0; i < j; ++i) {  // earlier rotations on the new column
                    const double a = H[size_t(i) * m + j], b = H[size_t(i + 1) * m + j];
                    H[size_t(i) * m + j] = cs[size_t(i)] * a + sn[size_t(i)] * b;
                    H[size_t(i + 1) * m + j] = -sn[size_t(i)] * a + cs[size_t(i)] * b;
                }
                const double a = H[size_t(j) * m + j], b = H[size_t(j + 1) * m + j];
                const double d = std::hypot(a, b);
                cs[size_t(j)] = d == 0.0 ? 1.0 : a / d;
                sn[size_t(j)] = d == 0.0 ? 0.0 : b / d;
                H[size_t(j) * m + j] = d;
                H[size_t(j + 1) * m + j] = 0.0;
                g[size_t(j) + 1] = -sn[size_t(j)] * g[size_t(j)];
                g[size_t(j)] = cs[size_t(j)] * g[size_t(j)];
                jj = j + 1;
                res.est_residual = std::fabs(g[size_t(j) + 1]) / fn;
                if (res.est_residual < rtol || it >= max_iter || d == 0.0)
                    break;
            }
            // least squares, then x += V y
            for (int i = jj - 1; i >= 0; --i) {
                double acc = g[size_t(i)];
                for (int c = i + 1; c < jj; ++c)
                    acc -= H[size_t(i) * m + c] * y[size_t(c)];
                y[size_t(i)] = acc / H[size_t(i) * m + i];
            }
            H3D_HIP(hipMemcpyAsync(hd, y.data(), sizeof(double) * size_t(jj),
                                   hipMemcpyHostToDevice, s));
            k_combine<<<gn, tb, 0, s>>>(n, V, n, jj, hd, 1.0, x);
            H3D_LAUNCH_CHECK();
            H3D_HIP(hipStreamSynchronize(s));
            res.cycles += 1;
        }
        res.iterations = it;
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    return res;
}

}  // namespace h3d
