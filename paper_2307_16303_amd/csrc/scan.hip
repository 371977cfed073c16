// Device-wide exclusive prefix sums (integer, so the result is exact and
// independent of the blocking).  1024 elements per workgroup, recursive over
// the per-workgroup totals.
#include "h3d_internal.hpp"

namespace h3d {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__global__ void __launch_bounds__(kScanThreads)
    k_scan_tile(const T *__restrict__ in, T *out, T *__restrict__ tile_sums, int64_t n) {
    __shared__ T sh[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(tid) * kScanItems;
    T v[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        v[k] = (base + k < n) ? in[base + k] : T(0);
    T tot = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        tot += v[k];
    sh[tid] = tot;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T add = (tid >= off) ? sh[tid - off] : T(0);
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    T run = sh[tid] - tot;  // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n)
            out[base + k] = run;
        run += v[k];
    }
    if (tid == kScanThreads - 1)
        tile_sums[blockIdx.x] = sh[tid];
}

template <typename T>
__global__ void k_scan_add(T *out, const T *__restrict__ tile_pre, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kScanTile + threadIdx.x;
    const T add = tile_pre[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t j = i + int64_t(k) * kScanThreads;
        if (j < n)
            out[j] += add;
    }
}

// exclusive scan of n values; tile totals of the top level go to total_out (device)
template <typename T>
void scan_rec(Plan &P, const T *in, T *out, int64_t n, T *total_out, hipStream_t s) {
    int64_t tiles = ceil_div(n, kScanTile);
    if (tiles < 1)
        tiles = 1;
    T *sums = P.mem.alloc_n<T>(tiles + 1);
    k_scan_tile<T><<<int(tiles), kScanThreads, 0, s>>>(in, out, sums, n);
    H3D_LAUNCH_CHECK();
    if (tiles == 1) {
        H3D_HIP(hipMemcpyAsync(total_out, sums, sizeof(T), hipMemcpyDeviceToDevice, s));
    } else {
        scan_rec<T>(P, sums, sums, tiles, total_out, s);
        k_scan_add<T><<<int(tiles), kScanThreads, 0, s>>>(out, sums, n);
        H3D_LAUNCH_CHECK();
    }
    H3D_HIP(hipStreamSynchronize(s));
    P.mem.release(sums);
}

}  // namespace

int64_t scan_exclusive_i64(Plan &P, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    if (n <= 0)
        return 0;
    int64_t *tot = P.mem.alloc_n<int64_t>(1);
    scan_rec<int64_t>(P, in, out, n, tot, s);
    int64_t h = 0;
    to_host(&h, tot, 1, s);
    P.mem.release(tot);
    return h;
}

void scan_exclusive_i32_nototal(Plan &P, const int32_t *in, int32_t *out, int64_t n,
                                hipStream_t s) {
    if (n <= 0)
        return;
    int32_t *tot = P.mem.alloc_n<int32_t>(1);
    scan_rec<int32_t>(P, in, out, n, tot, s);
    P.mem.release(tot);
}

}  // namespace h3d
