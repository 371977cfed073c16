// Factor construction: ACA in bounded FP64 workspace batches, then packing of
// each batch into the stored dtype (FP64, FP32, or BF16 with one FP32 scale per
// factor), and the column tables the mat-vec kernels stream by.
//
// Storage: a chunk per batch holds U_b (m x k, column-major) of its blocks in
// block order, then V_b (n x k).  Blocks of one target box are consecutive, so
// the columns of all U_b of a box form one m x (sum k) matrix whenever they
// land in the same chunk; every kernel nevertheless addresses factors through
// the per-block pointers, so a box may straddle chunks.
#include "h3d_internal.hpp"

namespace h3d {

void aca_level_batch(Plan &P, int level, const int32_t *list, int64_t q0, int64_t q1, double *ws,
                     const int64_t *ws_off, int64_t ws_base, int kws, int32_t *overflow,
                     unsigned int *ncapped, hipStream_t s);
void aca_workspace_sizes(Plan &P, const int32_t *list, int64_t cnt, int kws, int64_t *ws,
                         hipStream_t s);
void aca_pivot_sizes(Plan &P, int64_t *kc2, hipStream_t s);
void truncate_batch(Plan &P, const int32_t *list, int64_t q0, int64_t q1, int kws, double *ws,
                    const int64_t *ws_off, int64_t ws_base, const int32_t *overflow,
                    hipStream_t s);

namespace {

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return uint16_t((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);           // round to nearest even
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ void k_pack_sizes(int64_t q0, int64_t q1, const int32_t *__restrict__ list,
                             const int32_t *__restrict__ m, const int32_t *__restrict__ n,
                             const int32_t *__restrict__ rank, int64_t *__restrict__ mk,
                             int64_t *__restrict__ nk) {
    int64_t q = q0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= q1)
        return;
    const int64_t b = list[q];
    mk[q - q0] = int64_t(m[b]) * rank[b];
    nk[q - q0] = int64_t(n[b]) * rank[b];
}

__global__ void k_iota(int64_t n, int32_t *__restrict__ v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        v[i] = int32_t(i);
}

__global__ void k_flag_i64(int64_t n, const int32_t *__restrict__ flag, int64_t *__restrict__ out) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = flag[i] ? 1 : 0;
}

// deterministic compaction of the flagged blocks (ascending block order)
__global__ void k_compact(int64_t n, const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                          int32_t *__restrict__ list) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && flag[i])
        list[pos[i]] = int32_t(i);
}

template <int DT>
__global__ void __launch_bounds__(256)
    k_pack(int64_t q0, int64_t q1, const int32_t *__restrict__ list, const int32_t *__restrict__ m,
           const int32_t *__restrict__ n, const int32_t *__restrict__ rank, int max_rank, int kws,
           const double *__restrict__ ws, const int64_t *__restrict__ ws_off, int64_t ws_base,
           const int64_t *__restrict__ uoff, const int64_t *__restrict__ voff, char *cu, char *cv,
           void **uptr, void **vptr, float *scale2, int64_t panel_end,
           const int32_t *__restrict__ toff, const int32_t *__restrict__ leaf_off,
           const int32_t *__restrict__ leaf_of, int shc) {
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
    const int64_t nu = int64_t(mb) * k, nv = int64_t(nb) * k;
    const int64_t ou = uoff[q - q0], ov = voff[q - q0];
    // destination of element e (column-major index) of U_b: row panels above
    // the chunk level, column-major otherwise
    const bool panel = b < panel_end;
    const int32_t bs = toff[b];
    auto udst = [&](int64_t e) -> int64_t {
        if (!panel)
            return e;
        const int c = int(e / mb);
        return panel_off(leaf_off, leaf_of, shc, bs, k, int32_t(e - int64_t(c) * mb), c);
    };
    if (DT == H3D_F64) {
        double *du = reinterpret_cast<double *>(cu) + ou;
        double *dv = reinterpret_cast<double *>(cv) + ov;
        for (int64_t e = lane; e < nu; e += 64)
            du[udst(e)] = U[e];
        for (int64_t e = lane; e < nv; e += 64)
            dv[e] = V[e];
        if (lane == 0) {
            uptr[b] = du;
            vptr[b] = dv;
        }
    } else if (DT == H3D_F32) {
        float *du = reinterpret_cast<float *>(cu) + ou;
        float *dv = reinterpret_cast<float *>(cv) + ov;
        for (int64_t e = lane; e < nu; e += 64)
            du[udst(e)] = float(U[e]);
        for (int64_t e = lane; e < nv; e += 64)
            dv[e] = float(V[e]);
        if (lane == 0) {
            uptr[b] = du;
            vptr[b] = dv;
        }
    } else {
        uint16_t *du = reinterpret_cast<uint16_t *>(cu) + ou;
        uint16_t *dv = reinterpret_cast<uint16_t *>(cv) + ov;
        double su = 0.0, sv = 0.0;
        for (int64_t e = lane; e < nu; e += 64)
            su = fmax(su, fabs(U[e]));
        for (int64_t e = lane; e < nv; e += 64)
            sv = fmax(sv, fabs(V[e]));
        su = wave_max(su);
        sv = wave_max(sv);
        // the scales are powers of two, so dividing by them is exact
        su = su > 0.0 ? exp2(ceil(log2(su))) : 1.0;
        sv = sv > 0.0 ? exp2(ceil(log2(sv))) : 1.0;
        for (int64_t e = lane; e < nu; e += 64)
            du[udst(e)] = f32_to_bf16(float(U[e] / su));
        for (int64_t e = lane; e < nv; e += 64)
            dv[e] = f32_to_bf16(float(V[e] / sv));
        if (lane == 0) {
            uptr[b] = du;
            vptr[b] = dv;
            scale2[2 * b] = float(su);
            scale2[2 * b + 1] = float(sv);
        }
    }
}

__global__ void k_len_rank(int64_t nfar, const int32_t *__restrict__ len,
                           const int32_t *__restrict__ rank, int64_t *__restrict__ out) {
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b < nfar)
        out[b] = int64_t(len[b]) * rank[b];
}

__global__ void k_rank_i64(int64_t nfar, const int32_t *__restrict__ rank, int64_t *__restrict__ out) {
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b < nfar)
        out[b] = rank[b];
    if (b == nfar)
        out[b] = 0;
}

// stage-1 work items of the blocks [b0, b1) of one level; counts and offsets
// are indexed by b - b0
__global__ void k_item_count(int64_t b0, int64_t b1, int span, const int32_t *__restrict__ rank,
                             int64_t *__restrict__ cnt) {
    int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= b1)
        return;
    cnt[b - b0] = (rank[b] + span - 1) / span;
}

// split items: every column group of span columns is cut into parts of
// `rows` rows (enough parts for the longer of the two sides of the block);
// one reduction group per column group
__global__ void k_item_count_split(int64_t b0, int64_t b1, int span, int rows,
                                   const int32_t *__restrict__ m, const int32_t *__restrict__ n,
                                   const int32_t *__restrict__ rank, int64_t *__restrict__ cnt,
                                   int64_t *__restrict__ gcnt) {
    int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= b1)
        return;
    const int ncg = (rank[b] + span - 1) / span;
    const int np = max(1, (max(m[b], n[b]) + rows - 1) / rows);
    cnt[b - b0] = int64_t(ncg) * np;
    gcnt[b - b0] = ncg;
}

__global__ void k_item_fill_split(int64_t b0, int64_t b1, int span, int rows,
                                  const int32_t *__restrict__ m, const int32_t *__restrict__ n,
                                  const int32_t *__restrict__ rank, const int64_t *__restrict__ off,
                                  const int64_t *__restrict__ goff, int32_t *__restrict__ items,
                                  int32_t *__restrict__ part, int32_t *__restrict__ grp) {
    int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= b1)
        return;
    const int ncg = (rank[b] + span - 1) / span;
    const int np = max(1, (max(m[b], n[b]) + rows - 1) / rows);
    const int64_t o = off[b - b0], g = goff[b - b0];
    for (int q = 0; q < ncg; ++q) {
        grp[2 * (g + q)] = int32_t(o + int64_t(q) * np);
        grp[2 * (g + q) + 1] = np;
        for (int pp = 0; pp < np; ++pp) {
            const int64_t i = o + int64_t(q) * np + pp;
            items[2 * i] = int32_t(b);
            items[2 * i + 1] = q * span;
            part[i] = pp;
        }
    }
}

// packed items: the first block of every group of g consecutive blocks
// carries one item (first block, number of blocks)
__global__ void k_item_count_packed(int64_t b0, int64_t b1, int g, int64_t *__restrict__ cnt) {
    int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= b1)
        return;
    cnt[b - b0] = ((b - b0) % g) == 0 ? 1 : 0;
}

__global__ void k_item_fill_packed(int64_t b0, int64_t b1, int g, const int64_t *__restrict__ off,
                                   int32_t *__restrict__ items) {
    int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= b1 || ((b - b0) % g) != 0)
        return;
    const int64_t o = off[b - b0];
    items[2 * o] = int32_t(b);
    items[2 * o + 1] = int32_t(min<int64_t>(g, b1 - b));
}

__global__ void k_item_fill(int64_t b0, int64_t b1, int span, const int32_t *__restrict__ rank,
                            const int64_t *__restrict__ off, int32_t *__restrict__ items) {
    int64_t b = b0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= b1)
        return;
    const int64_t o = off[b - b0];
    for (int c = 0, q = 0; c < rank[b]; c += span, ++q) {
        items[2 * (o + q)] = int32_t(b);
        items[2 * (o + q) + 1] = c;
    }
}

// per-level sums of (m + n) k and of k, and the rank maximum
__global__ void k_level_sums(int64_t b0, int64_t b1, const int32_t *__restrict__ m,
                             const int32_t *__restrict__ n, const int32_t *__restrict__ rank,
                             unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[3][256];
    __shared__ unsigned int shm[256];
    unsigned long long e = 0, kk = 0, ev = 0;
    unsigned int mx = 0;
    for (int64_t b = b0 + int64_t(blockIdx.x) * 256 + threadIdx.x; b < b1;
         b += int64_t(gridDim.x) * 256) {
        e += (unsigned long long)(m[b] + n[b]) * (unsigned long long)rank[b];
        kk += (unsigned long long)rank[b];
        ev += (unsigned long long)n[b] * (unsigned long long)rank[b];
        mx = max(mx, (unsigned int)rank[b]);
    }
    sh[0][threadIdx.x] = e;
    sh[1][threadIdx.x] = kk;
    sh[2][threadIdx.x] = ev;
    shm[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + off];
            shm[threadIdx.x] = max(shm[threadIdx.x], shm[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], sh[0][0]);
        atomicAdd(&out[1], sh[1][0]);
        atomicMax(reinterpret_cast<unsigned int *>(&out[2]), shm[0]);
        atomicAdd(&out[3], sh[2][0]);
    }
}

template <int DT>
__global__ void __launch_bounds__(256)
    k_export(int64_t nfar, int which, const int32_t *__restrict__ len, const int32_t *__restrict__ rank,
             void *const *__restrict__ ptr, const float *__restrict__ scale2,
             const int64_t *__restrict__ off, double *__restrict__ out, int64_t panel_end,
             const int32_t *__restrict__ toff, const int32_t *__restrict__ leaf_off,
             const int32_t *__restrict__ leaf_of, int shc) {
    const int64_t b = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (b >= nfar)
        return;
    const int mb = len[b], k = rank[b];
    const int64_t cnt = int64_t(mb) * k;
    double *o = out + off[b];
    // source of element e (column-major index): row panels for U above the chunk level
    const bool panel = which == 0 && b < panel_end;
    const int32_t bs = toff[b];
    auto src = [&](int64_t e) -> int64_t {
        if (!panel)
            return e;
        const int c = int(e / mb);
        return panel_off(leaf_off, leaf_of, shc, bs, k, int32_t(e - int64_t(c) * mb), c);
    };
    if (DT == H3D_F64) {
        const double *p = reinterpret_cast<const double *>(ptr[b]);
        for (int64_t e = lane; e < cnt; e += 64)
            o[e] = p[src(e)];
    } else if (DT == H3D_F32) {
        const float *p = reinterpret_cast<const float *>(ptr[b]);
        for (int64_t e = lane; e < cnt; e += 64)
            o[e] = double(p[src(e)]);
    } else {
        const uint16_t *p = reinterpret_cast<const uint16_t *>(ptr[b]);
        const double sc = double(scale2[2 * b + which]);
        for (int64_t e = lane; e < cnt; e += 64)
            o[e] = double(bf16_to_f32(p[src(e)])) * sc;
    }
}

size_t dtype_size(int dt) { return dt == H3D_F64 ? 8 : (dt == H3D_F32 ? 4 : 2); }

}  // namespace

void factors_build(Plan &P, hipStream_t s) {
    const int64_t nf = P.nfar;
    const int dt = P.cfg.factor_dtype;
    P.factor_dtype = dt;
    // stage-2 chunk level: the deepest level whose boxes hold about 48 or
    // more points on average; U_b above it is stored as row panels
    int lc = P.L;
    while (lc > 0 && P.mean_box[lc] < 48)
        --lc;
    P.chunk_level = lc;
    P.panel_end = lc >= 1 ? P.lvl_blk[lc] : 0;
    const int shc = 3 * (P.L - lc);
    P.lu_form = (P.cfg.flags & H3D_FLAG_LU_FORM) != 0;
    P.blk_rank = P.mem.alloc_n<int32_t>(nf);
    P.blk_uptr = P.mem.alloc_n<void *>(nf);
    P.blk_vptr = P.mem.alloc_n<void *>(nf);
    if (P.lu_form) {
        // no explicit factors: the pointer tables stay NULL; one LU per block
        P.blk_lu = P.mem.alloc_n<void *>(nf);
        H3D_HIP(hipMemsetAsync(P.blk_uptr, 0, sizeof(void *) * size_t(nf), s));
        H3D_HIP(hipMemsetAsync(P.blk_vptr, 0, sizeof(void *) * size_t(nf), s));
        H3D_HIP(hipMemsetAsync(P.blk_lu, 0, sizeof(void *) * size_t(nf), s));
        P.leaf_fuse = 0;
    }
    P.blk_col0 = P.mem.alloc_n<int64_t>(nf + 1);
    if (dt == H3D_BF16_SCALED)
        P.blk_scale = P.mem.alloc_n<float>(2 * nf);
    if (nf == 0) {
        P.ncols = 0;
        H3D_HIP(hipMemsetAsync(P.blk_col0, 0, sizeof(int64_t), s));
        return;
    }
    H3D_HIP(hipMemsetAsync(P.blk_rank, 0, sizeof(int32_t) * size_t(nf), s));

    // the pivot + LU form needs the pivots (its build releases them unless kept)
    const bool keep_piv = (P.cfg.flags & H3D_FLAG_KEEP_PIVOTS) != 0 || P.lu_form;
    if (keep_piv) {
        int64_t *kc2 = P.mem.alloc_n<int64_t>(nf + 1);
        H3D_HIP(hipMemsetAsync(kc2 + nf, 0, sizeof(int64_t), s));
        aca_pivot_sizes(P, kc2, s);
        const int64_t tot = scan_exclusive_i64(P, kc2, kc2, nf + 1, s);
        P.blk_pivoff = kc2;
        P.blk_piv = P.mem.alloc_n<int32_t>(tot);
    }
    const int64_t budget0 =
        (P.cfg.workspace_bytes > 0 ? P.cfg.workspace_bytes : (int64_t(4) << 30)) / 8;
    unsigned int *ncapped = P.mem.alloc_n<unsigned int>(1);
    H3D_HIP(hipMemsetAsync(ncapped, 0, sizeof(unsigned int), s));
    int32_t *overflow = P.mem.alloc_n<int32_t>(nf);
    H3D_HIP(hipMemsetAsync(overflow, 0, sizeof(int32_t) * size_t(nf), s));
    int64_t *mk = P.mem.alloc_n<int64_t>(nf + 1);
    int64_t *nk = P.mem.alloc_n<int64_t>(nf + 1);
    int64_t *ws_off = P.mem.alloc_n<int64_t>(nf + 1);
    int32_t *list = P.mem.alloc_n<int32_t>(nf);
    k_iota<<<grid_for(nf, 256), 256, 0, s>>>(nf, list);
    H3D_LAUNCH_CHECK();
    int64_t cnt = nf;
    const size_t es = dtype_size(dt);
    hipEvent_t ev0, ev1;
    H3D_HIP(hipEventCreate(&ev0));
    H3D_HIP(hipEventCreate(&ev1));
    double aca_ms = 0.0;

    // Passes with a growing workspace column cap: a block stopped by the cap
    // before finishing is run again from the start with four times the room.
    // ACA is deterministic, so the result equals one run with unlimited room.
    for (int kws = 128; cnt > 0; kws = kws >= (1 << 28) ? kws : kws * 4) {
        H3D_HIP(hipMemsetAsync(ws_off + cnt, 0, sizeof(int64_t), s));
        aca_workspace_sizes(P, list, cnt, kws, ws_off, s);
        const int64_t ws_total = scan_exclusive_i64(P, ws_off, ws_off, cnt + 1, s);
        std::vector<int64_t> h_ws(size_t(cnt) + 1);
        std::vector<int32_t> h_list(static_cast<size_t>(cnt));
        to_host(h_ws.data(), ws_off, cnt + 1, s);
        to_host(h_list.data(), list, cnt, s);
        int64_t largest = 0;
        for (int64_t q = 0; q < cnt; ++q)
            largest = std::max(largest, h_ws[size_t(q) + 1] - h_ws[size_t(q)]);
        const int64_t budget = std::min(std::max(budget0, largest), ws_total);
        double *ws = P.mem.alloc_n<double>(budget);
        int64_t q0 = 0;
        while (q0 < cnt) {
            int64_t q1 = q0 + 1;
            while (q1 < cnt && h_ws[size_t(q1) + 1] - h_ws[size_t(q0)] <= budget)
                ++q1;
            const int64_t base = h_ws[size_t(q0)];
            H3D_HIP(hipEventRecord(ev0, s));
            for (int l = 1; l <= P.L; ++l) {
                // the list is in block order: find this level's positions
                const auto lo = std::lower_bound(h_list.begin() + q0, h_list.begin() + q1,
                                                 int32_t(P.lvl_blk[l]));
                const auto hi = std::lower_bound(lo, h_list.begin() + q1, int32_t(P.lvl_blk[l + 1]));
                const int64_t a = lo - h_list.begin(), e = hi - h_list.begin();
                if (e > a)
                    aca_level_batch(P, l, list, a, e, ws, ws_off, base, kws, overflow, ncapped, s);
            }
            H3D_HIP(hipEventRecord(ev1, s));
            H3D_HIP(hipEventSynchronize(ev1));
            float ms = 0.f;
            H3D_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            aca_ms += ms;
            // optional FP64 recompression to the optimal rank at tol
            if (P.cfg.flags & H3D_FLAG_TRUNCATE)
                truncate_batch(P, list, q0, q1, kws, ws, ws_off, base, overflow, s);
            // pack the finished blocks of the batch into their own chunk
            const int64_t nb = q1 - q0;
            if (P.lu_form) {
                lu_pack_batch(P, list, q0, q1, kws, ws, ws_off, base, mk, s);
                H3D_HIP(hipStreamSynchronize(s));
                q0 = q1;
                continue;
            }
            k_pack_sizes<<<grid_for(nb, 256), 256, 0, s>>>(q0, q1, list, P.blk_m, P.blk_n,
                                                           P.blk_rank, mk, nk);
            H3D_LAUNCH_CHECK();
            H3D_HIP(hipMemsetAsync(mk + nb, 0, sizeof(int64_t), s));
            H3D_HIP(hipMemsetAsync(nk + nb, 0, sizeof(int64_t), s));
            const int64_t tu = scan_exclusive_i64(P, mk, mk, nb + 1, s);
            const int64_t tv = scan_exclusive_i64(P, nk, nk, nb + 1, s);
            if (tu + tv > 0) {
                const size_t ubytes = (size_t(tu) * es + 255) & ~size_t(255);
                char *chunk = static_cast<char *>(P.mem.alloc(ubytes + size_t(tv) * es + 256));
                P.chunks.push_back(chunk);
                char *cu = chunk, *cv = chunk + ubytes;
                const int grid = grid_for(nb * 64, 256);
                const int mr = P.cfg.max_rank;
                switch (dt) {
                case H3D_F64:
                    k_pack<H3D_F64><<<grid, 256, 0, s>>>(q0, q1, list, P.blk_m, P.blk_n, P.blk_rank, mr,
                                                         kws, ws, ws_off, base, mk, nk, cu, cv,
                                                         P.blk_uptr, P.blk_vptr, P.blk_scale,
                                                         P.panel_end, P.blk_toff, P.leaf_off,
                                                         P.leaf_of, shc);
                    break;
                case H3D_F32:
                    k_pack<H3D_F32><<<grid, 256, 0, s>>>(q0, q1, list, P.blk_m, P.blk_n, P.blk_rank, mr,
                                                         kws, ws, ws_off, base, mk, nk, cu, cv,
                                                         P.blk_uptr, P.blk_vptr, P.blk_scale,
                                                         P.panel_end, P.blk_toff, P.leaf_off,
                                                         P.leaf_of, shc);
                    break;
                default:
                    k_pack<H3D_BF16_SCALED><<<grid, 256, 0, s>>>(
                        q0, q1, list, P.blk_m, P.blk_n, P.blk_rank, mr, kws, ws, ws_off, base, mk,
                        nk, cu, cv, P.blk_uptr, P.blk_vptr, P.blk_scale, P.panel_end, P.blk_toff,
                        P.leaf_off, P.leaf_of, shc);
                    break;
                }
                H3D_LAUNCH_CHECK();
            }
            H3D_HIP(hipStreamSynchronize(s));
            q0 = q1;
        }
        P.mem.release(ws);
        // blocks to run again
        int64_t *pos = mk;  // reuse as scan buffer of nf + 1 entries
        k_flag_i64<<<grid_for(nf, 256), 256, 0, s>>>(nf, overflow, pos);
        H3D_LAUNCH_CHECK();
        H3D_HIP(hipMemsetAsync(pos + nf, 0, sizeof(int64_t), s));
        // only listed blocks can have the flag set; others were cleared before
        cnt = scan_exclusive_i64(P, pos, pos, nf + 1, s);
        if (cnt > 0) {
            k_compact<<<grid_for(nf, 256), 256, 0, s>>>(nf, overflow, pos, list);
            H3D_LAUNCH_CHECK();
            H3D_HIP(hipMemsetAsync(overflow, 0, sizeof(int32_t) * size_t(nf), s));
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    P.stats.aca_ms = aca_ms;
    unsigned int hcap = 0;
    to_host(&hcap, ncapped, 1, s);
    P.stats.n_rank_capped = hcap;
    P.mem.release(ncapped);
    P.mem.release(overflow);
    P.mem.release(mk);
    P.mem.release(nk);
    P.mem.release(ws_off);
    P.mem.release(list);

    // factor columns: z index of every block, owner of every column
    k_rank_i64<<<grid_for(nf + 1, 256), 256, 0, s>>>(nf, P.blk_rank, P.blk_col0);
    H3D_LAUNCH_CHECK();
    P.ncols = scan_exclusive_i64(P, P.blk_col0, P.blk_col0, nf + 1, s);
    for (int l = 1; l <= P.L + 1 && l <= kMaxLevels; ++l) {
        int64_t v = 0;
        to_host(&v, P.blk_col0 + P.lvl_blk[l], 1, s);
        P.lvl_col[l] = v;
    }

    // statistics
    unsigned long long *sums = P.mem.alloc_n<unsigned long long>(4);
    int64_t entries = 0, bytes = 0, ev_total = 0;
    int rmax = 0;
    for (int l = 1; l <= P.L; ++l) {
        H3D_HIP(hipMemsetAsync(sums, 0, 4 * sizeof(unsigned long long), s));
        const int64_t lb = P.lvl_blk[l], le = P.lvl_blk[l + 1];
        if (le > lb) {
            k_level_sums<<<int(std::min<int64_t>(1024, ceil_div(le - lb, 256))), 256, 0, s>>>(
                lb, le, P.blk_m, P.blk_n, P.blk_rank, sums);
            H3D_LAUNCH_CHECK();
        }
        unsigned long long h[4];
        to_host(h, sums, 4, s);
        entries += int64_t(h[0]);
        ev_total += int64_t(h[3]);
        P.lvl_entries_v[l] = int64_t(h[3]);
        P.lvl_rank_sum[l] = int64_t(h[1]);
        P.lvl_entries_u[l] = int64_t(h[0]) - int64_t(h[3]);
        const int64_t lbytes = int64_t(h[0]) * int64_t(es) +
                               (dt == H3D_BF16_SCALED ? (le - lb) * 8 : 0);
        P.stats.factor_bytes_per_level[l] = lbytes;
        bytes += lbytes;
        rmax = std::max(rmax, int(uint32_t(h[2])));
    }
    P.mem.release(sums);
    P.stats.factor_entries = entries;
    P.entries_v = ev_total;
    P.stats.factor_bytes = bytes;
    P.stats.rank_sum = P.ncols;
    P.stats.rank_max = rmax;
    if (P.lu_form) {
        // pivot rows, the adjoint's column order and the work items; the
        // stored bytes are recounted there
        lu_finish(P, s);
        return;
    }

    // adjoint stage-1 items of the panelled levels
    for (int l = 1; l < P.chunk_level; ++l) {
        const int64_t b0 = P.lvl_blk[l], b1 = P.lvl_blk[l + 1];
        if (b1 <= b0)
            continue;
        const int64_t nb = b1 - b0;
        int64_t *cnt = P.mem.alloc_n<int64_t>(nb + 1);
        H3D_HIP(hipMemsetAsync(cnt + nb, 0, sizeof(int64_t), s));
        k_item_count<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, 8, P.blk_rank, cnt);
        H3D_LAUNCH_CHECK();
        const int64_t ni = scan_exclusive_i64(P, cnt, cnt, nb + 1, s);
        int32_t *items = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(ni, 1));
        k_item_fill<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, 8, P.blk_rank, cnt, items);
        H3D_LAUNCH_CHECK();
        H3D_HIP(hipStreamSynchronize(s));
        P.mem.release(cnt);
        P.s1a_items[l] = items;
        P.s1a_nitems[l] = ni;
    }

    // stage-1 shapes and work items (defaults; the autotuner may replace them)
    for (int cls = 0; cls < 2; ++cls)
        for (int l = 1; l <= P.L; ++l)
            set_level_shape(P, cls, l, default_shape(P, l, cls), s);
}

// Default stage-1 shape of level l: about four rows per lane, several tiny
// blocks per wave, and long columns split into single-pass items.
S1Shape default_shape(const Plan &P, int l, int cls) {
    const int m = P.mean_box[l];
    S1Shape sh;
    if (m <= 12) {
        sh.packed = 1;
        sh.S = 4;
        sh.U = 4;
    } else if (m <= 24) {
        sh.packed = 1;
        sh.S = 8;
        sh.U = 4;
    } else if (m <= 96) {
        sh.S = 16;
        sh.U = 4;
        sh.reps = 64;
    } else {
        sh.S = 64;
        sh.U = cls == 0 ? 8 : 4;
        sh.reps = m > 2048 ? 1 : 64;
    }
    return sh;
}

// (Re)builds the work items of level l for shape sh.
void set_level_shape(Plan &P, int cls, int l, const S1Shape &sh, hipStream_t s) {
    const int64_t b0 = P.lvl_blk[l], b1 = P.lvl_blk[l + 1];
    P.s1_shape[cls][l] = sh;
    P.mem.release(P.s1_items[cls][l]);
    P.s1_items[cls][l] = nullptr;
    P.s1_nitems[cls][l] = 0;
    if (cls == 0) {
        P.mem.release(P.s1_part[l]);
        P.mem.release(P.s1_grp[l]);
        P.mem.release(P.s1_zp[l]);
        P.s1_part[l] = P.s1_grp[l] = nullptr;
        P.s1_zp[l] = nullptr;
        P.s1_ngrp[l] = 0;
    }
    if (b1 <= b0)
        return;
    const int64_t nb = b1 - b0;
    if (!sh.packed && sh.rows > 0) {
        if (cls != 0)
            fail(H3D_EINVAL, "internal: split stage-1 shapes serve one right-hand side");
        const int span = (64 / sh.S) * sh.U;
        int64_t *cnt = P.mem.alloc_n<int64_t>(nb + 1);
        int64_t *gcnt = P.mem.alloc_n<int64_t>(nb + 1);
        H3D_HIP(hipMemsetAsync(cnt + nb, 0, sizeof(int64_t), s));
        H3D_HIP(hipMemsetAsync(gcnt + nb, 0, sizeof(int64_t), s));
        k_item_count_split<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, span, sh.rows, P.blk_m,
                                                             P.blk_n, P.blk_rank, cnt, gcnt);
        H3D_LAUNCH_CHECK();
        const int64_t ni = scan_exclusive_i64(P, cnt, cnt, nb + 1, s);
        const int64_t ng = scan_exclusive_i64(P, gcnt, gcnt, nb + 1, s);
        if (ni >= int64_t(0x7fffffff))
            fail(H3D_EINVAL, "too many stage-1 work items");
        int32_t *items = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(ni, 1));
        int32_t *part = P.mem.alloc_n<int32_t>(std::max<int64_t>(ni, 1));
        int32_t *grp = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(ng, 1));
        k_item_fill_split<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, span, sh.rows, P.blk_m, P.blk_n,
                                                            P.blk_rank, cnt, gcnt, items, part, grp);
        H3D_LAUNCH_CHECK();
        H3D_HIP(hipStreamSynchronize(s));
        P.mem.release(cnt);
        P.mem.release(gcnt);
        P.s1_items[0][l] = items;
        P.s1_nitems[0][l] = ni;
        P.s1_span[0][l] = span;
        P.s1_part[l] = part;
        P.s1_grp[l] = grp;
        P.s1_ngrp[l] = ng;
        P.s1_zp[l] = P.mem.alloc_n<double>(std::max<int64_t>(ni, 1) * span);
        return;
    }
    int64_t *cnt = P.mem.alloc_n<int64_t>(nb + 1);
    H3D_HIP(hipMemsetAsync(cnt + nb, 0, sizeof(int64_t), s));
    int span = 0;
    if (sh.packed) {
        k_item_count_packed<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, 64 / sh.S, cnt);
    } else {
        span = (64 / sh.S) * sh.U * std::max(1, sh.reps);
        k_item_count<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, span, P.blk_rank, cnt);
    }
    H3D_LAUNCH_CHECK();
    const int64_t ni = scan_exclusive_i64(P, cnt, cnt, nb + 1, s);
    int32_t *items = P.mem.alloc_n<int32_t>(2 * std::max<int64_t>(ni, 1));
    if (sh.packed)
        k_item_fill_packed<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, 64 / sh.S, cnt, items);
    else
        k_item_fill<<<grid_for(nb, 256), 256, 0, s>>>(b0, b1, span, P.blk_rank, cnt, items);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipStreamSynchronize(s));
    P.mem.release(cnt);
    P.s1_items[cls][l] = items;
    P.s1_nitems[cls][l] = ni;
    P.s1_span[cls][l] = span;
}

// Copies U (which = 0) or V (which = 1) of every block to host as FP64.
void export_factors(const Plan &Pc, int which, double *host_out) {
    Plan &P = const_cast<Plan &>(Pc);
    hipStream_t s = nullptr;
    const int64_t nf = P.nfar;
    if (nf == 0)
        return;
    const int32_t *len = which == 0 ? P.blk_m : P.blk_n;
    int64_t *off = P.mem.alloc_n<int64_t>(nf + 1);
    H3D_HIP(hipMemsetAsync(off + nf, 0, sizeof(int64_t), s));
    k_len_rank<<<grid_for(nf, 256), 256, 0, s>>>(nf, len, P.blk_rank, off);
    H3D_LAUNCH_CHECK();
    const int64_t tot = scan_exclusive_i64(P, off, off, nf + 1, s);
    double *out = P.mem.alloc_n<double>(tot);
    void *const *ptr = which == 0 ? P.blk_uptr : P.blk_vptr;
    const int grid = grid_for(nf * 64, 256);
    switch (P.factor_dtype) {
    case H3D_F64:
        k_export<H3D_F64><<<grid, 256, 0, s>>>(nf, which, len, P.blk_rank, ptr, P.blk_scale, off, out,
                                               P.panel_end, P.blk_toff, P.leaf_off, P.leaf_of,
                                               3 * (P.L - P.chunk_level));
        break;
    case H3D_F32:
        k_export<H3D_F32><<<grid, 256, 0, s>>>(nf, which, len, P.blk_rank, ptr, P.blk_scale, off, out,
                                               P.panel_end, P.blk_toff, P.leaf_off, P.leaf_of,
                                               3 * (P.L - P.chunk_level));
        break;
    default:
        k_export<H3D_BF16_SCALED><<<grid, 256, 0, s>>>(nf, which, len, P.blk_rank, ptr, P.blk_scale,
                                                       off, out, P.panel_end, P.blk_toff,
                                                       P.leaf_off, P.leaf_of,
                                                       3 * (P.L - P.chunk_level));
        break;
    }
    H3D_LAUNCH_CHECK();
    to_host(host_out, out, tot, s);
    P.mem.release(out);
    P.mem.release(off);
}

}  // namespace h3d
