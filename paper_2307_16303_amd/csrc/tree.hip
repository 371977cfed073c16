// Octree build (Sec. 2.1; depth rule of Algorithm 1): bounding cube, Morton
// keys, depth selection, leaf offsets and a stable bucket sort of the points.
//
// Quantisation is exact integer work derived from one FP64 product per axis:
// q21 = floor((x - lo) * 2^21 / side), clamped to [0, 2^21 - 1].  Because
// 2^21/side and 2^l/side differ by an exact power of two, q21 >> (21 - l)
// equals floor((x - lo) * 2^l / side) for every level l, so a single key per
// point serves all levels.  Boxes are half-open; the upper face is clamped
// into the last box.
#include "h3d_internal.hpp"

#pragma clang fp contract(off)

namespace h3d {

namespace {

constexpr int kQBits = 21;

__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint32_t quant21(double x, double lo, double scale) {
    double t = floor((x - lo) * scale);
    if (!(t >= 0.0))
        return 0u;
    if (t >= 2097152.0)
        return 2097151u;
    return uint32_t(t);
}

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

// per-workgroup min/max of each axis, count of non-finite coordinates and of
// points outside [lo, lo + side] (when check_box)
__global__ void __launch_bounds__(kRedThreads)
    k_bbox(const double *__restrict__ pts, int64_t n, int check_box, double lo0, double lo1,
           double lo2, double side, double *__restrict__ part, unsigned long long *__restrict__ bad) {
    __shared__ double smin[3][kRedThreads], smax[3][kRedThreads];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    unsigned long long nbad = 0, nout = 0;
    const double lo[3] = {lo0, lo1, lo2};
    for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kRedThreads) {
        for (int a = 0; a < 3; ++a) {
            double v = pts[3 * i + a];
            if (!isfinite(v)) {
                ++nbad;
                continue;
            }
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
            if (check_box && (v < lo[a] || v > lo[a] + side))
                ++nout;
        }
    }
    for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = mn[a];
        smax[a][threadIdx.x] = mx[a];
    }
    if (nbad)
        atomicAdd(&bad[0], nbad);
    if (nout)
        atomicAdd(&bad[1], nout);
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + off]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            part[6 * blockIdx.x + a] = smin[a][0];
            part[6 * blockIdx.x + 3 + a] = smax[a][0];
        }
}

__global__ void k_keys(const double *__restrict__ pts, int64_t n, double lo0, double lo1, double lo2,
                       double scale21, uint64_t *__restrict__ keys) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint64_t qx = quant21(pts[3 * i + 0], lo0, scale21);
    uint64_t qy = quant21(pts[3 * i + 1], lo1, scale21);
    uint64_t qz = quant21(pts[3 * i + 2], lo2, scale21);
    keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

__global__ void k_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                       uint32_t *__restrict__ bins) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    atomicAdd(&bins[keys[i] >> shift], 1u);
}

__global__ void __launch_bounds__(kRedThreads)
    k_max_u32(const uint32_t *__restrict__ v, int64_t n, uint32_t *__restrict__ part) {
    __shared__ uint32_t sh[kRedThreads];
    uint32_t m = 0;
    for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kRedThreads)
        m = max(m, v[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sh[0];
}

__global__ void k_u32_to_i32(const uint32_t *__restrict__ a, int32_t *__restrict__ b, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        b[i] = int32_t(a[i]);
}

// place every point in its leaf bucket (arbitrary order inside the bucket)
__global__ void k_scatter(const uint64_t *__restrict__ keys, int64_t n, int shift,
                          int32_t *__restrict__ cursor, int32_t *__restrict__ bucket) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int32_t pos = atomicAdd(&cursor[keys[i] >> shift], 1);
    bucket[pos] = int32_t(i);
}

// Sort each leaf bucket by original index: the rank of an element among the
// distinct indices of its bucket is its final position.  One wave per leaf.
__global__ void __launch_bounds__(256)
    k_leaf_sort(const int32_t *__restrict__ leaf_off, int64_t nleaf,
                const int32_t *__restrict__ bucket, int32_t *__restrict__ perm) {
    const int64_t leaf = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (leaf >= nleaf)
        return;
    const int32_t a = leaf_off[leaf], b = leaf_off[leaf + 1];
    for (int32_t e = a + lane; e < b; e += 64) {
        const int32_t v = bucket[e];
        int32_t rank = 0;
        for (int32_t f = a; f < b; ++f)
            rank += bucket[f] < v;
        perm[a + rank] = v;
    }
}

__global__ void k_gather_points(const double *__restrict__ pts, const int32_t *__restrict__ perm,
                                const uint64_t *__restrict__ keys, int64_t n, int shift,
                                double *__restrict__ px, double *__restrict__ py,
                                double *__restrict__ pz, int32_t *__restrict__ leaf_of) {
    int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    int64_t i = perm[p];
    px[p] = pts[3 * i + 0];
    py[p] = pts[3 * i + 1];
    pz[p] = pts[3 * i + 2];
    leaf_of[p] = int32_t(keys[i] >> shift);
}

}  // namespace

void tree_build(Plan &P, const double *pts, hipStream_t s) {
    const int64_t n = P.n;
    const h3d_config &c = P.cfg;
    const int check_box = c.box_side > 0.0;

    // bounding cube and validation of the coordinates
    {
        int nb = int(std::min<int64_t>(kRedBlocks, ceil_div(n, kRedThreads)));
        double *part = P.mem.alloc_n<double>(6 * nb);
        unsigned long long *bad = P.mem.alloc_n<unsigned long long>(2);
        H3D_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(unsigned long long), s));
        k_bbox<<<nb, kRedThreads, 0, s>>>(pts, n, check_box, c.box_lo[0], c.box_lo[1],
                                          c.box_lo[2], c.box_side, part, bad);
        H3D_LAUNCH_CHECK();
        std::vector<double> hp(6 * size_t(nb));
        unsigned long long hb[2];
        to_host(hp.data(), part, 6 * nb, s);
        to_host(hb, bad, 2, s);
        P.mem.release(part);
        P.mem.release(bad);
        if (hb[0])
            fail(H3D_EINVAL, std::to_string(hb[0]) + " non-finite point coordinates");
        if (hb[1])
            fail(H3D_EINVAL, std::to_string(hb[1]) + " coordinates outside the given box");
        if (check_box) {
            for (int a = 0; a < 3; ++a)
                P.lo[a] = c.box_lo[a];
            P.side = c.box_side;
        } else {
            double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int b = 0; b < nb; ++b)
                for (int a = 0; a < 3; ++a) {
                    mn[a] = std::min(mn[a], hp[6 * b + a]);
                    mx[a] = std::max(mx[a], hp[6 * b + 3 + a]);
                }
            double side = 0.0;
            for (int a = 0; a < 3; ++a) {
                P.lo[a] = mn[a];
                side = std::max(side, mx[a] - mn[a]);
            }
            P.side = side > 0.0 ? side : 1.0;
        }
    }

    // Morton keys at 21 bits per axis
    uint64_t *keys = P.mem.alloc_n<uint64_t>(n);
    const double scale21 = std::ldexp(1.0, kQBits) / P.side;
    k_keys<<<grid_for(n, 256), 256, 0, s>>>(pts, n, P.lo[0], P.lo[1], P.lo[2], scale21, keys);
    H3D_LAUNCH_CHECK();

    // depth rule: the smallest l whose boxes all hold at most leaf_size points
    int l0 = 0;
    while (l0 < c.max_depth && pow8(l0) * int64_t(c.leaf_size) < n)
        ++l0;
    int L = -1;
    uint32_t *bins = nullptr;
    for (int l = l0; l <= c.max_depth; ++l) {
        const int64_t nb = pow8(l);
        bins = P.mem.alloc_n<uint32_t>(nb);
        H3D_HIP(hipMemsetAsync(bins, 0, sizeof(uint32_t) * size_t(nb), s));
        k_hist<<<grid_for(n, 256), 256, 0, s>>>(keys, n, 3 * (kQBits - l), bins);
        H3D_LAUNCH_CHECK();
        int nred = int(std::min<int64_t>(kRedBlocks, ceil_div(nb, kRedThreads)));
        uint32_t *part = P.mem.alloc_n<uint32_t>(nred);
        k_max_u32<<<nred, kRedThreads, 0, s>>>(bins, nb, part);
        H3D_LAUNCH_CHECK();
        std::vector<uint32_t> hp(nred);
        to_host(hp.data(), part, nred, s);
        P.mem.release(part);
        uint32_t mx = 0;
        for (auto v : hp)
            mx = std::max(mx, v);
        if (int64_t(mx) <= int64_t(c.leaf_size)) {
            L = l;
            break;
        }
        P.mem.release(bins);
        bins = nullptr;
    }
    if (L < 0) {
        P.mem.release(keys);
        fail(H3D_EDEPTH, "no depth <= " + std::to_string(c.max_depth) +
                             " gives leaves of at most " + std::to_string(c.leaf_size) + " points");
    }
    P.L = L;
    const int64_t nleaf = pow8(L);
    const int shift = 3 * (kQBits - L);

    // leaf offsets
    int32_t *counts = P.mem.alloc_n<int32_t>(nleaf + 1);
    k_u32_to_i32<<<grid_for(nleaf, 256), 256, 0, s>>>(bins, counts, nleaf);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipMemsetAsync(counts + nleaf, 0, sizeof(int32_t), s));
    P.mem.release(bins);
    P.leaf_off = P.mem.alloc_n<int32_t>(nleaf + 1);
    scan_exclusive_i32_nototal(P, counts, P.leaf_off, nleaf + 1, s);
    P.mem.release(counts);

    // stable order inside leaves: bucket by leaf, then rank by original index
    int32_t *cursor = P.mem.alloc_n<int32_t>(nleaf);
    H3D_HIP(hipMemcpyAsync(cursor, P.leaf_off, sizeof(int32_t) * size_t(nleaf),
                           hipMemcpyDeviceToDevice, s));
    int32_t *bucket = P.mem.alloc_n<int32_t>(n);
    k_scatter<<<grid_for(n, 256), 256, 0, s>>>(keys, n, shift, cursor, bucket);
    H3D_LAUNCH_CHECK();
    P.perm = P.mem.alloc_n<int32_t>(n);
    k_leaf_sort<<<grid_for(nleaf * 64, 256), 256, 0, s>>>(P.leaf_off, nleaf, bucket, P.perm);
    H3D_LAUNCH_CHECK();
    P.px = P.mem.alloc_n<double>(n);
    P.py = P.mem.alloc_n<double>(n);
    P.pz = P.mem.alloc_n<double>(n);
    P.leaf_of = P.mem.alloc_n<int32_t>(n);
    k_gather_points<<<grid_for(n, 256), 256, 0, s>>>(pts, P.perm, keys, n, shift, P.px, P.py,
                                                     P.pz, P.leaf_of);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipStreamSynchronize(s));
    P.mem.release(cursor);
    P.mem.release(bucket);
    P.mem.release(keys);

    P.h_leaf_off.resize(size_t(nleaf) + 1);
    to_host(P.h_leaf_off.data(), P.leaf_off, nleaf + 1, s);
}

}  // namespace h3d
