// HODLR3D mat-vec (Algorithm 2) and its adjoint on the device.
//
//   gather   xp = x[perm]                               (sorted order)
//   near     yn_t = sum_{s in Near(t)} K(t,s) xp_s      (leaf blocks, kernel
//            entries evaluated on the fly, sources staged through LDS)
//   stage 1  z_b = V_b^T xp_s  for every far block b    (factor stream; in the
//            adjoint U_b^T xp_t)
//   stage 2  y_t = yn_t + sum_levels sum_{b of t} U_b z_b, written straight
//            to y[perm] (in the adjoint V_b z_b summed over the blocks whose
//            source is the box)
//   with one right-hand side the finest level may instead run both stages at
//   once (leaf.hip), adding its far field into yn before stage 2 runs over
//   the coarser levels
//
// Stage 1 treats every factor column as one dot product: a sub-wave of S
// lanes (S ~ the level's box size) walks one column, so 64/S consecutive
// columns, which are consecutive in memory, are read per wave instruction.
// Stage 2 gives every row its own lane (two rows for boxes of 65..128 points):
// one workgroup per box of a chunk level (boxes of roughly 64 points), looping
// over the levels; at each level the lane streams the column slices of the
// factors of the box that contains its row.  No atomics: every output row is
// written by exactly one lane, and the summation order is fixed, so results
// are bitwise reproducible.
#include <unistd.h>

#include <cmath>
#include <cstdlib>

#include "stage1_items.hpp"

namespace h3d {

namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// per-phase kernels of one operator
__global__ void k_gather(const void *__restrict__ x, int io_f32, int64_t ldx, int64_t n, int nrhs,
                         const int32_t *__restrict__ perm, double *__restrict__ xp) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n)
        gather_row(x, io_f32, ldx, n, nrhs, perm, xp, p);
}

// near field: one wave per leaf (KIND: the kernel fixed at compile time, or -1)
template <int NR, bool E32, int KIND>
__global__ void __launch_bounds__(64)
    k_near(const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ near_ptr,
           const int32_t *__restrict__ near_s, const double *__restrict__ px,
           const double *__restrict__ py, const double *__restrict__ pz, int kind, double kp,
           int nrhs, const double *__restrict__ xp, int64_t n, double *__restrict__ yn) {
    near_leaf<NR, E32, KIND>(blockIdx.x, leaf_off, near_ptr, near_s, px, py, pz, kind, kp,
                                    nrhs, xp, n, yn);
}

// Workgroups are dealt to the eight XCDs in turn (each XCD with its own L2).
// Workgroup b is renumbered so that every XCD takes a contiguous run of the
// grid: consecutive work items, whose factors lie back to back and share the
// cache line at their common end, then meet in one L2.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t nwg) {
    const int64_t q = nwg >> 3, r = nwg & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// stage 1: one work item per wave
template <int S, int U, int DT, int NR>
__global__ void __launch_bounds__(256) k_s1_wide(S1Args a) {
    const int64_t b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t w = uniform64((b * blockDim.x + threadIdx.x) >> 6);
    if (w < a.nitems)
        s1_wide_item<S, U, DT, NR>(a, w);
}

template <int S, int U, int DT, int NR>
__global__ void __launch_bounds__(256) k_s1_packed(S1Args a) {
    const int64_t b = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t w = uniform64((b * blockDim.x + threadIdx.x) >> 6);
    if (w < a.nitems)
        s1_packed_item<S, U, DT, NR>(a, w);
}

// split columns: z of every column group = its parts' partial sums, added in
// part order (one thread per column of a group)
__global__ void __launch_bounds__(256)
    k_s1_reduce(int64_t ngrp, const int32_t *__restrict__ grp, S1Args a) {
    s1_reduce_column(int64_t(blockIdx.x) * blockDim.x + threadIdx.x, ngrp, grp, a);
}

// one launch of level l's stage 1 with its current shape
template <int DT, int NR> void launch_s1(const S1Shape &sh, S1Args a, hipStream_t s) {
    const int grid = grid_for(a.nitems * 64, 256);
    if (sh.packed) {
#define H3D_S1P(SS, UU)                                                                   \
    if (sh.S == SS && sh.U == UU) {                                                       \
        k_s1_packed<SS, UU, DT, NR><<<grid, 256, 0, s>>>(a);                              \
        return;                                                                           \
    }
        H3D_S1P(4, 2) H3D_S1P(4, 4) H3D_S1P(8, 2) H3D_S1P(8, 4) H3D_S1P(16, 2) H3D_S1P(16, 4)
        // narrow factors, one right-hand side: twice the loads in flight
        if constexpr (NR == 1 && DT != H3D_F64) {
            H3D_S1P(4, 8) H3D_S1P(8, 8) H3D_S1P(16, 8)
        }
#undef H3D_S1P
    } else {
#define H3D_S1W(SS, UU)                                                                   \
    if (sh.S == SS && sh.U == UU) {                                                       \
        k_s1_wide<SS, UU, DT, NR><<<grid, 256, 0, s>>>(a);                                \
        return;                                                                           \
    }
        H3D_S1W(8, 4) H3D_S1W(8, 8) H3D_S1W(16, 4) H3D_S1W(16, 8) H3D_S1W(32, 4) H3D_S1W(32, 8)
        H3D_S1W(64, 2) H3D_S1W(64, 4) H3D_S1W(64, 8)
        if constexpr (NR == 1 && DT != H3D_F64) {
            H3D_S1W(16, 16) H3D_S1W(32, 16) H3D_S1W(64, 16)
        }
#undef H3D_S1W
    }
    fail(H3D_EDEVICE, "internal: no stage-1 kernel for this shape");
}

// level l's stage 1 with its current shape, including the reduction of split
// columns
template <int DT, int NR>
void launch_s1_level(const Plan &P, int l, const S1Shape &sh, const S1Args &a, hipStream_t s) {
    launch_s1<DT, NR>(sh, a, s);
    if (a.part) {
        H3D_LAUNCH_CHECK();
        const int64_t nt = P.s1_ngrp[l] * a.span;
        k_s1_reduce<<<grid_for(nt, 256), 256, 0, s>>>(P.s1_ngrp[l], P.s1_grp[l], a);
    }
}

// adjoint stage 1 of a panelled level: one work item per wave
template <int DT, int NR>
__global__ void __launch_bounds__(256)
    k_s1_panel(S1Args a, const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ box,
               int shc, int shl) {
    const int64_t w = uniform64((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
    if (w < a.nitems)
        s1_panel_item<DT, NR>(a, leaf_off, box, shc, shl, w);
}

// stage 2: one workgroup per chunk box.  Neighbouring chunk boxes share the
// cache line at their common edge in every coarse column they read, and
// workgroups are dealt to the eight XCDs (each with its own L2) in turn: each
// XCD gets a contiguous run of chunk boxes so that those lines are fetched once.
// (FP64 factors, one RHS: at most 128 registers, four waves per SIMD, which
// the compiler reaches without spilling)
template <int DT, int NR, int kS2Waves>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(DT == H3D_F64 && NR == 1 ? 4 : 1)))
    k_stage2(S2Tab tab, const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ leaf_of,
             const int64_t *__restrict__ grp_begin, const int64_t *__restrict__ grp_blk,
             void *const *__restrict__ fptr, const int32_t *__restrict__ rank,
             const int64_t *__restrict__ blk_col0, const double *__restrict__ z, int64_t ldz,
             const double *yn, int64_t n, int nrhs, const int32_t *__restrict__ perm,
             void *__restrict__ yout, int64_t ldy, int io_f32, int lb, int le, double *ypart) {
    const int64_t nch = gridDim.x;
    int64_t B = blockIdx.x;
    if ((nch & 7) == 0)
        B = (B & 7) * (nch >> 3) + (B >> 3);
    stage2_chunk<DT, NR, kS2Waves>(B, tab, leaf_off, leaf_of, grp_begin, grp_blk, fptr, rank,
                                   blk_col0, z, ldz, yn, n, nrhs, perm, yout, ldy, io_f32, lb, le,
                                   ypart);
}

template <int DT, int NR>
void launch_s2_kernel(int waves, int64_t nchunk, hipStream_t s, const S2Tab &tab, const Plan &P,
                      const int64_t *grp_blk, void *const *fptr, const double *z, const double *yn,
                      int nrhs, void *y, int64_t ldy, int io_f32, int lb, int le, double *ypart) {
#define H3D_S2(W)                                                                           \
    k_stage2<DT, NR, W><<<int(nchunk), 64 * W, 0, s>>>(                                     \
        tab, P.leaf_off, P.leaf_of, P.tgt_begin, grp_blk, fptr, P.blk_rank, P.blk_col0, z,  \
        P.ncols, yn, P.n, nrhs, P.perm, y, ldy, io_f32, lb, le, ypart)
    if (waves <= 1)
        H3D_S2(1);
    else if (waves <= 2)
        H3D_S2(2);
    else if (waves <= 4)
        H3D_S2(4);
    else
        H3D_S2(8);
#undef H3D_S2
    H3D_LAUNCH_CHECK();
}

template <int DT, int NR>
S1Args stage1_args(const Plan &P, int cls, int l, bool adjoint, int nrhs, const double *xp,
                   double *z) {
    S1Args a{};
    a.items = reinterpret_cast<const int2 *>(P.s1_items[cls][l]);
    a.nitems = P.s1_nitems[cls][l];
    a.span = P.s1_span[cls][l];
    a.blk_col0 = P.blk_col0;
    a.rank = P.blk_rank;
    a.seg_len = adjoint ? P.blk_m : P.blk_n;
    a.seg_off = adjoint ? P.blk_toff : P.blk_soff;
    a.seg_ptr = adjoint ? P.blk_uptr : P.blk_vptr;
    a.scale2 = P.blk_scale;
    a.nrhs = nrhs;
    a.xp = xp;
    a.n = P.n;
    a.z = z;
    a.ldz = P.ncols;
    if (cls == 0 && P.s1_part[l]) {
        a.part = P.s1_part[l];
        a.rows = P.s1_shape[0][l].rows;
        a.zp = P.s1_zp[l];
    }
    return a;
}

template <int DT, int NR>
void launch_far(Plan &P, bool adjoint, int nrhs, const double *xp, double *z, const double *yn,
                void *y, int64_t ldy, int io_f32, hipStream_t s) {
    const int64_t n = P.n;
    const int L = P.L;
    const int cls = NR == 1 ? 0 : 1;
    const double es = DT == H3D_F64 ? 8.0 : (DT == H3D_F32 ? 4.0 : 2.0);
    // one right-hand side: the finest level may run both stages in k_leaf
    const int leaf_sh = NR == 1 ? leaf_shape(P) : 0;
    const int Lf = leaf_sh ? L - 1 : L;  // last level of the two-stage form
    // stage 1: one launch per level
    for (int l = 1; l <= Lf; ++l) {
        const S1Args a = stage1_args<DT, NR>(P, cls, l, adjoint, nrhs, xp, z);
        if (a.nitems == 0)
            continue;
        const S1Shape &sh = P.s1_shape[cls][l];
        const double ent = double(adjoint ? P.lvl_entries_u[l] : P.lvl_entries_v[l]);
        const double cols = double(P.lvl_rank_sum[l]);
        const double bytes = ent * es + cols * 8.0 * nrhs + double(n) * 8.0 * nrhs;
        // the adjoint reads U_b, stored as row panels above the chunk level
        const bool pan = adjoint && l < P.chunk_level;
        hipEvent_t ev = P.prof.begin(s);
        if (pan) {
            S1Args ap = a;
            ap.items = reinterpret_cast<const int2 *>(P.s1a_items[l]);
            ap.nitems = P.s1a_nitems[l];
            ap.span = kPanelCols;
            k_s1_panel<DT, NR><<<grid_for(ap.nitems * 64, 256), 256, 0, s>>>(
                ap, P.leaf_off, P.blk_t, 3 * (L - P.chunk_level), 3 * (P.chunk_level - l));
        } else {
            launch_s1_level<DT, NR>(P, l, sh, a, s);
        }
        H3D_LAUNCH_CHECK();
        const char *kname = pan ? "k_s1_panel" : (sh.packed ? "k_s1_packed" : "k_s1_wide");
        char name[48];
        if (P.prof.levels)
            snprintf(name, sizeof(name), "%s_L%d", kname, l);
        else
            snprintf(name, sizeof(name), "%s", kname);
        P.prof.end(s, ev, name, bytes, 2.0 * ent * nrhs);
    }
    if (leaf_sh) {
        const double ent = double(P.lvl_entries_u[L] + P.lvl_entries_v[L]);
        const double bytes = ent * es + double(P.n) * 24.0;
        hipEvent_t ev = P.prof.begin(s);
        launch_leaf(P, leaf_sh, adjoint, xp, const_cast<double *>(yn), s);
        char name[48];
        snprintf(name, sizeof(name), P.prof.levels ? "k_leaf_L%d" : "k_leaf", L);
        P.prof.end(s, ev, name, bytes, 4.0 * ent);
    }
    // stage 2 (always: it also writes y); level by level when profiling
    // levels, carrying the partial sums in yn
    S2Tab tab{};
    for (int l = 0; l <= kMaxLevels; ++l)
        tab.box_base[l] = P.box_base[l];
    tab.L = L;
    tab.lc = P.chunk_level;
    tab.panel = adjoint ? 0 : 1;
    const int64_t nchunk = pow8(P.chunk_level);
    const int parts = (P.prof.levels && Lf > 1) ? Lf : 1;
    for (int part = 1; part <= parts; ++part) {
        const int lb = parts == 1 ? 1 : part, le = parts == 1 ? Lf : part;
        const bool last = part == parts;
        double ent = double(adjoint ? P.entries_v : P.stats.factor_entries - P.entries_v);
        double cols = double(P.ncols);
        if (leaf_sh) {
            ent -= double(adjoint ? P.lvl_entries_v[L] : P.lvl_entries_u[L]);
            cols -= double(P.lvl_rank_sum[L]);
        }
        if (parts > 1) {
            ent = double(adjoint ? P.lvl_entries_v[part] : P.lvl_entries_u[part]);
            cols = double(P.lvl_rank_sum[part]);
        }
        const double bytes = ent * es + cols * 8.0 * nrhs +
                             double(n) * (8.0 + (io_f32 ? 4.0 : 8.0)) * nrhs + double(n) * 8.0;
        hipEvent_t ev = P.prof.begin(s);
        launch_s2_kernel<DT, NR>(P.s2_waves[cls], nchunk, s, tab, P, adjoint ? P.src_blk : nullptr,
                                 adjoint ? P.blk_vptr : P.blk_uptr, z, yn, nrhs, y, ldy, io_f32,
                                 lb, le, last ? nullptr : const_cast<double *>(yn));
        char name[48];
        if (parts > 1)
            snprintf(name, sizeof(name), "k_stage2_L%d", part);
        else
            snprintf(name, sizeof(name), "k_stage2");
        P.prof.end(s, ev, name, bytes, 2.0 * ent * nrhs);
    }
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate stage-1 shapes level by level and stage-2 wave
// counts on the plan's own factor streams, keeps the fastest of each.
std::vector<S1Shape> s1_candidates(const Plan &P, int l, bool narrow, bool split) {
    std::vector<S1Shape> c;
    const int m = std::max(1, P.mean_box[l]);
    auto add = [&](int packed, int S, int U, int reps) {
        S1Shape sh;
        sh.packed = packed;
        sh.S = S;
        sh.U = U;
        sh.reps = reps;
        c.push_back(sh);
    };
    if (m <= 32) {
        add(1, 4, 2, 1);
        add(1, 4, 4, 1);
        add(1, 8, 2, 1);
        add(1, 8, 4, 1);
        if (narrow) {
            add(1, 4, 8, 1);
            add(1, 8, 8, 1);
        }
    }
    if (m >= 8 && m <= 128) {
        add(1, 16, 2, 1);
        add(1, 16, 4, 1);
        if (narrow)
            add(1, 16, 8, 1);
    }
    for (int S : {8, 16, 32, 64}) {
        if (S > std::max(8, 2 * m) || 16 * S < m)
            continue;
        for (int U : {4, 8}) {
            add(0, S, U, 1);
            add(0, S, U, 64);
        }
        if (S == 64)
            add(0, 64, 2, 1);
        if (narrow && S >= 16) {
            add(0, S, 16, 1);
            add(0, S, 16, 64);
        }
    }
    // long columns, one right-hand side: split into parts of `rows` rows
    if (split && m > 512)
        for (int rows : {512, 2048})
            for (int U : {4, 8, 16}) {
                if (U == 16 && !narrow)
                    continue;
                add(0, 64, U, 1);
                c.back().rows = rows;
            }
    return c;
}

template <int DT, int NR>
void autotune_dt(Plan &P, int nrhs, hipStream_t s) {
    const int cls = NR == 1 ? 0 : 1;
    hipEvent_t e0, e1;
    H3D_HIP(hipEventCreate(&e0));
    H3D_HIP(hipEventCreate(&e1));
    auto time_it = [&](auto &&launch) {
        launch();  // warm-up
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            H3D_HIP(hipEventRecord(e0, s));
            launch();
            H3D_HIP(hipEventRecord(e1, s));
            H3D_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            H3D_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return best;
    };
    for (int l = 1; l <= P.L; ++l) {
        if (P.lvl_blk[l + 1] <= P.lvl_blk[l])
            continue;
        S1Shape best_sh = P.s1_shape[cls][l];
        float best_ms = 1e30f;
        for (const S1Shape &sh : s1_candidates(P, l, NR == 1 && DT != H3D_F64, NR == 1)) {
            set_level_shape(P, cls, l, sh, s);
            const S1Args a = stage1_args<DT, NR>(P, cls, l, false, nrhs, P.xp, P.z);
            const float ms = time_it([&] { launch_s1_level<DT, NR>(P, l, sh, a, s); });
            if (ms < best_ms) {
                best_ms = ms;
                best_sh = sh;
            }
        }
        set_level_shape(P, cls, l, best_sh, s);
    }
    // one right-hand side: the finest level fused (S lanes per column) or not,
    // timed over the whole far field
    if (NR == 1 && !P.in_batch && P.lvl_blk[P.L + 1] > P.lvl_blk[P.L]) {
        int best_s = 0;
        float best_f = 1e30f;
        for (int S : leaf_candidates()) {
            P.leaf_fuse = S;
            const float ms = time_it([&] {
                launch_far<DT, 1>(P, false, 1, P.xp, P.z, P.yp, P.yp + P.n, P.n, 0, s);
            });
            if (ms < best_f) {
                best_f = ms;
                best_s = S;
            }
        }
        P.leaf_fuse = best_s;
    }
    // stage-2 waves per chunk box, timed on the levels stage 2 covers once the
    // finest level is settled
    S2Tab tab{};
    for (int l = 0; l <= kMaxLevels; ++l)
        tab.box_base[l] = P.box_base[l];
    tab.L = P.L;
    tab.lc = P.chunk_level;
    tab.panel = 1;
    const int64_t nchunk = pow8(P.chunk_level);
    const int Lf = NR == 1 && leaf_shape(P) ? P.L - 1 : P.L;
    float best_ms = 1e30f;
    int best_w = P.s2_waves[cls];
    for (int w : {2, 4, 8}) {
        const float ms = time_it([&] {
            launch_s2_kernel<DT, NR>(w, nchunk, s, tab, P, nullptr, P.blk_uptr, P.z, P.yp, nrhs,
                                     P.yp + P.n * nrhs, P.n, 0, 1, Lf, nullptr);
        });
        if (ms < best_ms) {
            best_ms = ms;
            best_w = w;
        }
    }
    P.s2_waves[cls] = best_w;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P.tuned[cls] = true;
}

template <int NR>
void launch_near(Plan &P, int nrhs, const double *xp, double *yn, hipStream_t s) {
    hipEvent_t ev = P.prof.begin(s);
    // the FP32 and BF16 forms evaluate the near-field entries in FP32; the
    // Laplace kernel has launches of its own (the general ones inline every
    // kernel's formula)
    const int g = int(pow8(P.L));
    const bool e32 = P.factor_dtype != H3D_F64, lap = P.cfg.kernel == H3D_LAPLACE;
#define H3D_NEAR(E, K)                                                                      \
    k_near<NR, E, K><<<g, 64, 0, s>>>(P.leaf_off, P.near_ptr, P.near_s, P.px, P.py, P.pz,   \
                                      P.cfg.kernel, P.cfg.kernel_param, nrhs, xp, P.n, yn)
    if (e32) {
        if (lap)
            H3D_NEAR(true, H3D_LAPLACE);
        else
            H3D_NEAR(true, -1);
    } else {
        if (lap)
            H3D_NEAR(false, H3D_LAPLACE);
        else
            H3D_NEAR(false, -1);
    }
#undef H3D_NEAR
    H3D_LAUNCH_CHECK();
    P.prof.end(s, ev, "k_near", double(P.n) * (32.0 + 8.0 * nrhs),
               double(P.stats.near_pair_evals) * (10.0 + 2.0 * nrhs));
}

}  // namespace

void ensure_scratch(Plan &P, int64_t nrhs, hipStream_t s) {
    if (nrhs <= P.scratch_nrhs)
        return;
    const int64_t n = P.n;
    if (P.xp)
        before_release(P, "a product with more right-hand sides");
    P.mem.release(P.xp);
    P.mem.release(P.yp);
    P.mem.release(P.z);
    P.xp = P.mem.alloc_n<double>(n * nrhs);
    P.yp = P.mem.alloc_n<double>(2 * n * nrhs);  // second half: tuner output
    P.z = P.mem.alloc_n<double>(std::max<int64_t>(P.ncols, 1) * nrhs);
    H3D_HIP(hipMemsetAsync(P.xp, 0, sizeof(double) * size_t(n * nrhs), s));
    H3D_HIP(hipMemsetAsync(P.yp, 0, sizeof(double) * size_t(2 * n * nrhs), s));
    P.scratch_nrhs = nrhs;
}

// ---- the tuner's cache ------------------------------------------------------
// H3D_TUNE_CACHE names a JSON file mapping a plan's key (GPU architecture,
// factor type, one or several right-hand sides, depth, batch membership (a
// member does not fuse the finest level), and per level the
// half-octave buckets of the mean box size and the mean rank) to the shapes
// the tuner chose: [finest-level fusion, stage-2 waves, then per level
// packed, S, U, passes, rows].  A plan whose key is found takes the stored
// shapes (each checked against the level's candidates) instead of timing;
// otherwise the tuner runs and adds its result.  The file is rewritten whole,
// through a temporary file and a rename.

int half_octave(double v) { return v <= 0.0 ? -1 : int(std::floor(2.0 * std::log2(v))); }

std::string tune_key(const Plan &P, int cls) {
    hipDeviceProp_t prop{};
    H3D_HIP(hipGetDeviceProperties(&prop, P.device));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::string k = arch + "|dt" + std::to_string(P.factor_dtype) + "|nr" +
                    std::to_string(cls == 0 ? 1 : 4) + "|L" + std::to_string(P.L) +
                    (P.in_batch ? "|batch" : "");
    for (int l = 1; l <= P.L; ++l) {
        const int64_t nb = P.lvl_blk[l + 1] - P.lvl_blk[l];
        const double mr = nb > 0 ? double(P.lvl_rank_sum[l]) / double(nb) : 0.0;
        k += "|" + std::to_string(half_octave(P.mean_box[l])) + ":" +
             std::to_string(half_octave(mr));
    }
    return k;
}

std::map<std::string, std::vector<int>> read_tune_file(const char *path) {
    std::map<std::string, std::vector<int>> out;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0)
        text.append(buf, got);
    std::fclose(f);
    // entries: "key": [int, int, ...]
    size_t pos = 0;
    for (;;) {
        const size_t q0 = text.find('"', pos);
        if (q0 == std::string::npos)
            break;
        const size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos)
            break;
        const size_t b0 = text.find('[', q1);
        const size_t b1 = b0 == std::string::npos ? b0 : text.find(']', b0);
        if (b1 == std::string::npos)
            break;
        std::vector<int> v;
        const char *c = text.c_str() + b0 + 1;
        const char *e = text.c_str() + b1;
        while (c < e) {
            char *end = nullptr;
            const long x = std::strtol(c, &end, 10);
            if (end == c) {
                ++c;
                continue;
            }
            v.push_back(int(x));
            c = end;
        }
        out[text.substr(q0 + 1, q1 - q0 - 1)] = v;
        pos = b1 + 1;
    }
    return out;
}

void write_tune_file(const char *path, const std::map<std::string, std::vector<int>> &m) {
    const std::string tmp = std::string(path) + ".tmp." + std::to_string(long(getpid()));
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f)
        return;  // the cache is an optimisation: an unwritable path only costs tuning time
    std::fputs("{\n", f);
    size_t i = 0;
    for (const auto &kv : m) {
        std::fprintf(f, "  \"%s\": [", kv.first.c_str());
        for (size_t j = 0; j < kv.second.size(); ++j)
            std::fprintf(f, j ? ", %d" : "%d", kv.second[j]);
        std::fputs(++i < m.size() ? "],\n" : "]\n", f);
    }
    std::fputs("}\n", f);
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0)
        std::remove(tmp.c_str());
}

// applies a stored entry when every value is one the tuner could have chosen
bool tune_cache_apply(Plan &P, int cls, const std::vector<int> &v, bool narrow, hipStream_t s) {
    if (v.size() != size_t(2 + 5 * P.L))
        return false;
    const std::vector<int> lc = leaf_candidates();
    if (cls == 0 && std::find(lc.begin(), lc.end(), v[0]) == lc.end())
        return false;
    if (v[1] != 2 && v[1] != 4 && v[1] != 8)
        return false;
    std::vector<S1Shape> shapes(size_t(P.L) + 1);
    for (int l = 1; l <= P.L; ++l) {
        const int *e = v.data() + 2 + 5 * (l - 1);
        S1Shape sh;
        sh.packed = e[0];
        sh.S = e[1];
        sh.U = e[2];
        sh.reps = e[3];
        sh.rows = e[4];
        bool known = P.lvl_blk[l + 1] <= P.lvl_blk[l];  // empty levels keep any shape
        for (const S1Shape &c : s1_candidates(P, l, narrow, cls == 0))
            known = known || (c.packed == sh.packed && c.S == sh.S && c.U == sh.U &&
                              c.reps == sh.reps && c.rows == sh.rows);
        known = known || (sh.packed == P.s1_shape[cls][l].packed && sh.S == P.s1_shape[cls][l].S &&
                          sh.U == P.s1_shape[cls][l].U && sh.reps == P.s1_shape[cls][l].reps &&
                          sh.rows == P.s1_shape[cls][l].rows);
        if (!known)
            return false;
        shapes[size_t(l)] = sh;
    }
    for (int l = 1; l <= P.L; ++l)
        if (P.lvl_blk[l + 1] > P.lvl_blk[l])
            set_level_shape(P, cls, l, shapes[size_t(l)], s);
    if (cls == 0 && !P.in_batch)
        P.leaf_fuse = v[0];
    P.s2_waves[cls] = v[1];
    P.tuned[cls] = true;
    return true;
}

std::vector<int> tune_cache_entry(const Plan &P, int cls) {
    std::vector<int> v{cls == 0 ? std::max(P.leaf_fuse, 0) : 0, P.s2_waves[cls]};
    for (int l = 1; l <= P.L; ++l) {
        const S1Shape &sh = P.s1_shape[cls][l];
        v.insert(v.end(), {sh.packed, sh.S, sh.U, sh.reps, sh.rows});
    }
    return v;
}

void autotune(Plan &P, int64_t nrhs, hipStream_t s) {
    // the pivot + LU form has no launch shapes to choose
    if (P.nfar == 0 || nrhs >= kBatchedMinRhs || P.lu_form)
        return;
    // the tuner rebuilds the stage-1 work tables that earlier products used
    if (P.built)
        before_release(P, "autotuning");
    const int nr = nrhs == 1 ? 1 : int(std::min<int64_t>(nrhs, 4));
    ensure_scratch(P, std::max<int64_t>(nrhs, nr), s);
    const int cls = nrhs == 1 ? 0 : 1;
    const char *cache = std::getenv("H3D_TUNE_CACHE");
    std::string key;
    if (cache && *cache) {
        key = tune_key(P, cls);
        const auto m = read_tune_file(cache);
        const auto it = m.find(key);
        const bool narrow = nrhs == 1 && P.factor_dtype != H3D_F64;
        if (it != m.end() && tune_cache_apply(P, cls, it->second, narrow, s)) {
            H3D_HIP(hipStreamSynchronize(s));
            P.stats.tune_source = 2;
            return;
        }
    }
    auto go = [&](auto dt_tag) {
        constexpr int DT = decltype(dt_tag)::value;
        if (nrhs == 1)
            autotune_dt<DT, 1>(P, 1, s);
        else
            autotune_dt<DT, 4>(P, int(nrhs), s);
    };
    switch (P.factor_dtype) {
    case H3D_F64:
        go(std::integral_constant<int, H3D_F64>{});
        break;
    case H3D_F32:
        go(std::integral_constant<int, H3D_F32>{});
        break;
    default:
        go(std::integral_constant<int, H3D_BF16_SCALED>{});
        break;
    }
    H3D_HIP(hipStreamSynchronize(s));
    P.stats.tune_source = 1;
    if (cache && *cache) {
        auto m = read_tune_file(cache);
        m[key] = tune_cache_entry(P, cls);
        write_tune_file(cache, m);
    }
}

void launch_near_field(Plan &P, int nrhs, const double *xp, double *yn, hipStream_t s) {
    if (nrhs == 1)
        launch_near<1>(P, 1, xp, yn, s);
    else
        launch_near<4>(P, nrhs, xp, yn, s);
}

int64_t vector_z_entries(const Plan &P, int64_t nrhs) {
    // the pivot + LU form runs kLuGroup right-hand sides at a time
    if (P.lu_form)
        return std::max<int64_t>(P.ncols, 1) * std::min<int64_t>(nrhs, kLuGroup);
    // one right-hand side with the finest level fused: z of that level (the
    // last columns) is never stored
    if (nrhs == 1 && P.L >= 1 && leaf_shape(P))
        return std::max<int64_t>(P.lvl_col[P.L], 1);
    return std::max<int64_t>(P.ncols, 1) * nrhs;
}

void matvec_vector(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                   int io_dtype, bool adjoint, double *xp, double *yn, double *z, hipStream_t s) {
    const int64_t n = P.n;
    const int io_f32 = io_dtype == H3D_F32;
    if (P.lu_form) {
        // kLuGroup columns at a time through the same scratch
        const size_t es = io_f32 ? 4 : 8;
        for (int64_t c = 0; c < nrhs; c += kLuGroup)
            matvec_lu(P, static_cast<const char *>(x) + size_t(c * ldx) * es,
                      static_cast<char *>(y) + size_t(c * ldy) * es,
                      std::min<int64_t>(kLuGroup, nrhs - c), ldx, ldy, io_dtype, adjoint, xp, yn, z,
                      s);
        return;
    }
    {
        hipEvent_t ev = P.prof.begin(s);
        k_gather<<<grid_for(n, 256), 256, 0, s>>>(x, io_f32, ldx, n, int(nrhs), P.perm, xp);
        H3D_LAUNCH_CHECK();
        P.prof.end(s, ev, "k_gather", double(n) * (4.0 + (io_f32 ? 4.0 : 8.0) * nrhs + 8.0 * nrhs), 0.0);
    }
    // The near list is symmetric (t in Near(s) iff s in Near(t)), and the
    // kernels are radial, so K(t,s)^T = K(s,t): the adjoint near field walks
    // the same list with the roles of row and column exchanged.
    if (nrhs == 1)
        launch_near<1>(P, 1, xp, yn, s);
    else
        launch_near<4>(P, int(nrhs), xp, yn, s);
    auto far = [&](auto dt_tag) {
        constexpr int DT = decltype(dt_tag)::value;
        if (nrhs == 1)
            launch_far<DT, 1>(P, adjoint, 1, xp, z, yn, y, ldy, io_f32, s);
        else
            launch_far<DT, 4>(P, adjoint, int(nrhs), xp, z, yn, y, ldy, io_f32, s);
    };
    switch (P.factor_dtype) {
    case H3D_F64:
        far(std::integral_constant<int, H3D_F64>{});
        break;
    case H3D_F32:
        far(std::integral_constant<int, H3D_F32>{});
        break;
    default:
        far(std::integral_constant<int, H3D_BF16_SCALED>{});
        break;
    }
}

void matvec_run(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                int io_dtype, bool adjoint, hipStream_t s) {
    if (P.lu_form) {
        ensure_scratch(P, std::min<int64_t>(nrhs, kLuGroup), s);
        matvec_vector(P, x, y, nrhs, ldx, ldy, io_dtype, adjoint, P.xp, P.yp, P.z, s);
        return;
    }
    if (nrhs >= kBatchedMinRhs) {
        matvec_batched(P, x, y, nrhs, ldx, ldy, io_dtype, adjoint, s);
        return;
    }
    ensure_scratch(P, nrhs, s);
    matvec_vector(P, x, y, nrhs, ldx, ldy, io_dtype, adjoint, P.xp, P.yp, P.z, s);
}

}  // namespace h3d
