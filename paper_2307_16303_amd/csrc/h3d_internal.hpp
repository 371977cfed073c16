// Internal definitions of libhodlr3d: the plan (every device array of one
// HODLR3D operator), allocation, error handling and the kernel profiler.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hodlr3d.h"

namespace h3d {

struct Error : std::runtime_error {
    h3d_status code;
    Error(h3d_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(h3d_status c, const std::string &m) { throw Error(c, m); }

#define H3D_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            ::h3d::fail(e_ == hipErrorOutOfMemory ? H3D_ENOMEM : H3D_EDEVICE,              \
                        std::string(#call) + ": " + hipGetErrorString(e_));                \
    } while (0)

#define H3D_LAUNCH_CHECK() H3D_HIP(hipGetLastError())

constexpr int kMaxLevels = H3D_MAX_LEVELS;  // levels 0..10
constexpr int kMaxDepth = kMaxLevels - 1;

inline int64_t pow8(int l) { return int64_t(1) << (3 * l); }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device memory owned by a plan, obtained through the caller's allocator or
// hipMalloc.
class DeviceMemory {
  public:
    DeviceMemory() = default;
    DeviceMemory(const DeviceMemory &) = delete;
    DeviceMemory &operator=(const DeviceMemory &) = delete;
    ~DeviceMemory() { release_all(); }

    void configure(const h3d_allocator *a, hipStream_t s) {
        if (a && a->alloc && a->free) {
            user_ = *a;
            has_user_ = true;
        }
        stream_ = s;
    }
    void *alloc(size_t bytes) {
        if (bytes == 0)
            bytes = 8;
        bytes = (bytes + 255) & ~size_t(255);
        void *p = nullptr;
        if (has_user_) {
            p = user_.alloc(bytes, (void *)stream_, user_.ctx);
            if (!p)
                fail(H3D_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                fail(H3D_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
            }
        }
        live_[p] = bytes;
        total_ += bytes;
        return p;
    }
    template <typename T> T *alloc_n(int64_t n) { return (T *)alloc(size_t(n > 0 ? n : 1) * sizeof(T)); }
    void release(void *p) {
        if (!p)
            return;
        auto it = live_.find(p);
        if (it == live_.end())
            return;
        size_t bytes = it->second;
        live_.erase(it);
        total_ -= bytes;
        if (has_user_)
            user_.free(p, bytes, (void *)stream_, user_.ctx);
        else
            (void)hipFree(p);
    }
    void release_all() {
        while (!live_.empty())
            release(live_.begin()->first);
    }
    size_t total() const { return total_; }

  private:
    h3d_allocator user_{};
    bool has_user_ = false;
    hipStream_t stream_ = nullptr;
    std::map<void *, size_t> live_;
    size_t total_ = 0;
};

// HIP-event timing of the mat-vec kernels, per kernel name.
struct Profiler {
    bool on = false;
    bool levels = false;  // launch the factor streams level by level
    struct Rec {
        int slot;
        hipEvent_t a, b;
    };
    std::vector<std::string> names;
    std::vector<int64_t> launches;
    std::vector<double> total_ms, bytes, flops;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;

    int slot_of(const char *name) {
        for (size_t i = 0; i < names.size(); ++i)
            if (names[i] == name)
                return int(i);
        names.emplace_back(name);
        launches.push_back(0);
        total_ms.push_back(0.0);
        bytes.push_back(0.0);
        flops.push_back(0.0);
        return int(names.size() - 1);
    }
    hipEvent_t get_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        H3D_HIP(hipEventCreate(&e));
        return e;
    }
    // Brackets one launch: begin() before it, end() after it.
    hipEvent_t begin(hipStream_t s) {
        if (!on)
            return nullptr;
        hipEvent_t a = get_event();
        H3D_HIP(hipEventRecord(a, s));
        return a;
    }
    void end(hipStream_t s, hipEvent_t a, const char *name, double nbytes, double nflops) {
        if (!on || !a)
            return;
        hipEvent_t b = get_event();
        H3D_HIP(hipEventRecord(b, s));
        int slot = slot_of(name);
        bytes[slot] += nbytes;
        flops[slot] += nflops;
        pending.push_back({slot, a, b});
    }
    void collect() {
        for (auto &r : pending) {
            H3D_HIP(hipEventSynchronize(r.b));
            float ms = 0.f;
            H3D_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            launches[r.slot] += 1;
            total_ms[r.slot] += ms;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    void reset() {
        collect();
        for (size_t i = 0; i < names.size(); ++i) {
            launches[i] = 0;
            total_ms[i] = 0.0;
            bytes[i] = 0.0;
            flops[i] = 0.0;
        }
    }
    ~Profiler() {
        for (auto &r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool)
            (void)hipEventDestroy(e);
    }
};

// Shape of one level's stage-1 launch (see the stage-1 kernels).
struct S1Shape {
    int packed = 0;  // 1: one sub-wave per block, 64/S blocks per wave
    int S = 64;      // lanes per factor column
    int U = 8;       // columns in flight per lane and pass
    int reps = 1;    // wide form: passes per work item
    int rows = 0;    // wide form, one RHS: > 0 splits each column into parts of this
                     // many rows (partial sums, then a fixed-order reduction)
};

// Everything one HODLR3D operator owns.  Rows are numbered in sorted (Morton)
// order; a box b at level l owns rows leaf_off[b 8^(L-l)] .. leaf_off[(b+1) 8^(L-l)].
struct Plan {
    h3d_config cfg{};
    DeviceMemory mem;
    int device = 0;
    int64_t n = 0;
    int L = 0;
    double lo[3] = {0, 0, 0};
    double side = 1.0;

    // tree
    int32_t *perm = nullptr;      // [n] sorted row -> original index
    int32_t *iperm = nullptr;     // [n] original index -> sorted row (many-RHS tables)
    double *px = nullptr, *py = nullptr, *pz = nullptr;  // [n] sorted coordinates
    int32_t *leaf_off = nullptr;  // [8^L + 1]
    int32_t *leaf_of = nullptr;   // [n] leaf of each sorted row
    std::vector<int32_t> h_leaf_off;  // host copy

    // boxes of all levels 1..L concatenated: global box id g = box_base[l] + t
    int64_t box_base[kMaxLevels + 1] = {0};
    int64_t nbox_all = 0;

    // far blocks in (level, target, source) order
    int64_t nfar = 0;
    int64_t lvl_blk[kMaxLevels + 1] = {0};  // blocks of level l: [lvl_blk[l], lvl_blk[l+1])
    int64_t *tgt_begin = nullptr;  // [nbox_all + 1] blocks of global box g as target
    int64_t *src_blk = nullptr;    // [nfar] blocks grouped by source box (same offsets)
    int32_t *blk_t = nullptr, *blk_s = nullptr;        // box ids (per level)
    int32_t *blk_toff = nullptr, *blk_m = nullptr;     // target rows
    int32_t *blk_soff = nullptr, *blk_n = nullptr;     // source rows
    int32_t *blk_rank = nullptr;
    int64_t *blk_col0 = nullptr;   // first factor column (z index) of each block
    void **blk_uptr = nullptr;     // device pointer to U_b (m x k, column-major)
    void **blk_vptr = nullptr;     // device pointer to V_b (n x k, column-major)
    float *blk_scale = nullptr;    // BF16 form: scale of U_b times scale of V_b
    int32_t *blk_piv = nullptr;    // optional: 2 kcap ints per block
    int64_t *blk_pivoff = nullptr;
    int64_t ncols = 0;             // sum of ranks
    int64_t entries_v = 0;         // sum of n k (entries of all V_b)
    int64_t lvl_entries_u[kMaxLevels + 1] = {0};  // per level: sum of m k
    int64_t lvl_entries_v[kMaxLevels + 1] = {0};  // per level: sum of n k
    int64_t lvl_col[kMaxLevels + 1] = {0};
    // stage-1 launch shape and work items per level, for one right-hand side
    // (class 0) and for several (class 1)
    S1Shape s1_shape[2][kMaxLevels + 1];
    int32_t *s1_items[2][kMaxLevels + 1] = {};  // [2 count]: (block, c0) or (first, count)
    int64_t s1_nitems[2][kMaxLevels + 1] = {};
    int s1_span[2][kMaxLevels + 1] = {};        // wide form: columns per item
    // split levels (class 0): part index of every item, reduction groups
    // (first item, parts) of every (block, column group), partial sums
    int32_t *s1_part[kMaxLevels + 1] = {};
    int32_t *s1_grp[kMaxLevels + 1] = {};
    int64_t s1_ngrp[kMaxLevels + 1] = {};
    double *s1_zp[kMaxLevels + 1] = {};
    int s2_waves[2] = {4, 4};                    // waves per stage-2 chunk box
    int leaf_fuse = -1;  // one RHS: lanes per column of the fused finest level
                         // (0: not fused, -1: chosen from the leaf size)
    bool tuned[2] = {false, false};
    int64_t lvl_rank_sum[kMaxLevels + 1] = {0};
    int chunk_level = 0;           // stage-2 boxes: about 64 rows per wave
    int64_t panel_end = 0;         // blocks [0, panel_end) store U_b as row panels
    // adjoint stage-1 items of the panelled levels: (block, first of 8 columns)
    int32_t *s1a_items[kMaxLevels + 1] = {};
    int64_t s1a_nitems[kMaxLevels + 1] = {};
    int mean_box[kMaxLevels + 1] = {0};  // mean size of non-empty boxes per level
    int max_box[kMaxLevels + 1] = {0};

    // near field at the leaf level
    int64_t nnear = 0;
    int32_t *near_ptr = nullptr;  // [8^L + 1]
    int32_t *near_s = nullptr;    // [nnear]
    int8_t *near_rel = nullptr;   // [nnear]

    // stored factors
    int factor_dtype = H3D_F64;
    std::vector<void *> chunks;

    // the pivot + LU form (H3D_FLAG_LU_FORM, lu_form.hip): per block the packed
    // LU factors of K(sigma, tau); per factor column the sorted rows of its two
    // pivot points; the adjoint's column order (blocks grouped by source);
    // stage-1 work items and the partial sums of split blocks
    bool lu_form = false;
    void **blk_lu = nullptr;          // [nfar] k x k column-major
    int64_t lu_sq = 0;                // sum of k^2
    int32_t *lu_sig_row = nullptr;    // [ncols]
    int32_t *lu_tau_row = nullptr;    // [ncols]
    int64_t *lu_adj_col0 = nullptr;   // [nfar + 1] over the positions of src_blk
    int32_t *lu_adj_col = nullptr;    // [ncols]
    void *lu_items[2] = {};           // forward, adjoint
    int64_t lu_nitems[2] = {};
    void *lu_split[2] = {};
    int64_t lu_nsplit[2] = {};
    int64_t lu_wcols = 0;
    double *lu_wpart = nullptr;
    h3d_stats stats{};

    // mat-vec scratch, grown on demand
    int64_t scratch_nrhs = 0;
    double *xp = nullptr, *yp = nullptr, *z = nullptr;

    // many right-hand sides (matrix-core path): work items and point-major
    // scratch, built on first use
    bool bt_ready = false;
    int32_t *bt_near = nullptr;
    int64_t bt_nnear = 0;
    int32_t *bt_s1[kMaxLevels + 1] = {};
    int64_t bt_ns1[kMaxLevels + 1] = {};
    // FP32/BF16 stage 1: (block, column tile group), blocks in source order
    // (forward) and in level order (adjoint)
    int32_t *bt_s1r[kMaxLevels + 1][2] = {};
    int64_t bt_ns1r[kMaxLevels + 1][2] = {};
    int32_t *bt_s2r[kMaxLevels + 1] = {};  // FP32/BF16 stage 2: (box, 64-row tile)
    int64_t bt_ns2r[kMaxLevels + 1] = {};
    int32_t *bt_s2k[kMaxLevels + 1][2] = {};  // K-steps per box of the ring kernel (fwd, adj)
    int32_t *bt_s2k16[kMaxLevels + 1] = {};    // BF16 stage 2: K-steps of 16 columns per box
    int32_t *bt_pk[kMaxLevels + 1] = {};  // adjoint stage 1 above the chunk level: 16-row super-steps per box
    int bt_mt1[kMaxLevels + 1] = {};  // 16-column tiles per stage-1 wave
    int bt_split[kMaxLevels + 1] = {};  // stage-1 rows per part (0: columns not split)
    int32_t *bt_grp[kMaxLevels + 1] = {};  // split levels: (first item, parts) per tile
    int64_t bt_ngrp[kMaxLevels + 1] = {};
    void *bzp = nullptr;  // partial stage-1 tiles of the split levels
    size_t bzp_bytes = 0;
    // fused finest level for leaves of 17..64 rows (leaf_fused.hip): leaves
    // grouped by 16-row tile count
    bool lf_ready = false, lf_ok = false;
    int32_t *lf_items[4] = {};
    int64_t lf_n[4] = {};
    void *bx = nullptr, *by = nullptr, *bz = nullptr;
    size_t bx_bytes = 0, by_bytes = 0, bz_bytes = 0;
    void *bxh = nullptr;  // BF16 factors: x as BF16 hi/lo words (bf16_mfma.hip)
    size_t bxh_bytes = 0;

    Profiler prof;
    bool built = false;
    bool in_batch = false;  // a problem of a batch: launch shapes fixed
    // HIP graphs captured from this plan's products: they hold the device
    // addresses of the scratch and of the work tables, so while any exists
    // nothing that a product uses may be freed or reallocated
    int live_graphs = 0;
};

// Called before scratch or work tables that earlier products used are
// released to grow or rebuild them: refuses while a captured graph holds
// their addresses, then drains the device, so that no kernel of an earlier
// product on any stream still uses the memory when the allocator takes it
// back.
inline void before_release(Plan &P, const char *what) {
    if (P.live_graphs > 0)
        fail(H3D_EINVAL, std::string(what) + " would reallocate memory that " +
                             std::to_string(P.live_graphs) +
                             " captured graph(s) of this plan use: destroy them first");
    H3D_HIP(hipDeviceSynchronize());
}

// products with at least this many right-hand sides use the matrix cores
constexpr int64_t kBatchedMinRhs = 8;

// Fused finest level of a one-RHS product (leaf.hip): rows of an output leaf
// per pass, and the launch of shape (lanes per column) | (columns in flight
// << 8), adding the level's far field into the sorted sums yn.
constexpr int kLeafRows = 16;
void launch_leaf(const Plan &P, int shape, bool adjoint, const double *xp, double *yn,
                 hipStream_t s);
// the shape a one-RHS product of P uses (0: the finest level runs in the two
// stages), and the shapes the autotuner tries (0 among them)
int leaf_shape(const Plan &P);
std::vector<int> leaf_candidates();

// Row panels.  Stage 2 gives one workgroup to each box of the chunk level lc
// and streams, for every coarser level, the rows of U_b that fall in that
// box.  So the U_b of a block whose level lies above lc is stored as one
// panel per chunk box of its target box, in row order; a panel holds the
// chunk box's rows of all k columns, column-major (leading dimension = the
// chunk box's row count), so each workgroup reads one contiguous range.
// Blocks at or below lc keep U_b column-major (one panel).  V_b is always
// column-major.  Offset of element (i, c) of a panelled U_b whose target box
// starts at sorted row bs; shc = 3 (L - lc).
__device__ __forceinline__ int64_t panel_off(const int32_t *__restrict__ leaf_off,
                                             const int32_t *__restrict__ leaf_of, int shc,
                                             int32_t bs, int k, int32_t i, int c) {
    const int32_t row = bs + i;
    const int32_t ch = leaf_of[row] >> shc;
    const int32_t r0 = leaf_off[ch << shc], r1 = leaf_off[(ch + 1) << shc];
    return int64_t(r0 - bs) * k + (row - r0) + int64_t(c) * (r1 - r0);
}

struct BatchState;
}  // namespace h3d

// The opaque handle of the C ABI: one operator, or a batch of independent
// operators (then P holds only the batch's own device tables and profiler).
struct h3d_plan {
    h3d::Plan P;
    h3d::BatchState *batch = nullptr;
    ~h3d_plan();
};

namespace h3d {

struct BatchProb;  // device descriptor of one problem (batch.hip)
struct BatchSeg;   // a run of queue items of one kind and problem (batch.hip)

// A batch of independent operators multiplied together, one launch per phase
// over all problems.
struct BatchState {
    std::vector<h3d_plan *> subs;  // owned
    BatchProb *probs = nullptr;    // device [nprob]
    BatchSeg *segs = nullptr;      // device [nseg]
    int nseg = 0;
    int64_t nitems = 0;            // work items (units) over all launches
    // per launch: kind, shape (stage 2: waves), first and end segment, first
    // unit, units; [0] one right-hand side, [1] two to seven
    std::vector<int64_t> launches[2];
    const void **io = nullptr;     // device [2 nprob]: x pointers then y pointers
    int64_t desc_nrhs = 0;         // right-hand sides the descriptors were written for
    std::vector<const void *> desc_scratch;  // scratch pointers they hold
    ~BatchState() {
        for (h3d_plan *p : subs)
            delete p;
    }
};

void batch_setup(h3d_plan &batch, hipStream_t s);
void batch_run(h3d_plan &batch, const void *const *x, void *const *y, int64_t nrhs, int io_dtype,
               hipStream_t s);

// ---- building blocks implemented in the .hip files ----
void tree_build(Plan &P, const double *points, hipStream_t s);
void lists_build(Plan &P, hipStream_t s);
void factors_build(Plan &P, hipStream_t s);
void matvec_run(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                int io_dtype, bool adjoint, hipStream_t s);
// The product for nrhs < kBatchedMinRhs with caller-given scratch: xp and yn
// hold n nrhs doubles each, z vector_z_entries(P, nrhs).  Every value of the
// three is written before it is read, so none needs clearing.
void matvec_vector(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                   int io_dtype, bool adjoint, double *xp, double *yn, double *z, hipStream_t s);
int64_t vector_z_entries(const Plan &P, int64_t nrhs);
void export_factors(const Plan &P, int which, double *host_out);
void set_level_shape(Plan &P, int cls, int l, const S1Shape &sh, hipStream_t s);
S1Shape default_shape(const Plan &P, int l, int cls);
void autotune(Plan &P, int64_t nrhs, hipStream_t s);
// grows the plan's mat-vec scratch (xp, yp, z) to nrhs right-hand sides
void ensure_scratch(Plan &P, int64_t nrhs, hipStream_t s);
void matvec_batched(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
                    int io_dtype, bool adjoint, hipStream_t s);

// near field of a product (FP64 entries, or FP32 entries for FP32/BF16 factors)
void launch_near_field(Plan &P, int nrhs, const double *xp, double *yn, hipStream_t s);
// many right-hand sides, FP32/BF16 factors: both stages of the finest level
// in one pass per leaf for leaves of at most 64 rows (leaf_fused.hip)
bool leaf_fused_tables(Plan &P, hipStream_t s);
// stage 1 of one level (not split into row parts), FP32/BF16 factors, one
// wave per (block, 16 MT factor columns) with a ring of fragment loads
// (stage1_ring.hip); MT from the level's mean rank
int s1_ring_tiles(const Plan &P, int l);
void launch_s1_ring(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                    const float *Xs, int NP, float *Z, hipStream_t s);
// stage 2 of one level, FP32/BF16 factors, one wave per (box, 64-row tile)
// with a ring of fragment loads across the box's blocks (stage2_ring.hip)
// FP64 matrix-core ring kernels (stage_ring64.hip)
void launch_s1_ring64(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                      const double *Xs, int NP, double *Z, hipStream_t s);
void launch_s2_ring64(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                      const double *Z, int NP, double *Y, hipStream_t s);
// BF16 matrix-core stages (forward products with BF16 factors)
int32_t *s2_bf16_steps(Plan &P, int l, hipStream_t s);
void launch_split_x(const float *Xs, int64_t count, uint32_t *Xh, hipStream_t s);
void launch_s1_bf16(Plan &P, int l, const int2 *items, int64_t nitems, const uint32_t *Xh, int NP,
                    uint32_t *Zh, hipStream_t s);
void launch_s2_bf16(Plan &P, int l, const int2 *items, int64_t nitems, const uint32_t *Zh, int NP,
                    double *Y, hipStream_t s);
// per box of level l (above the chunk level), the K-steps of its row panels
int32_t *panel_steps(Plan &P, int l, hipStream_t s);
// per box of level l, the K-steps of its blocks in the stage-2 ring kernel
int32_t *s2_ring_steps(Plan &P, int l, bool adjoint, hipStream_t s);
void launch_s2_ring(Plan &P, int l, bool adjoint, const int2 *items, int64_t nitems,
                    const float *Z, int NP, double *Y, hipStream_t s);
void launch_leaf_fused(Plan &P, const float *Xs, int NP, double *Y, bool adjoint, hipStream_t s);
// many-RHS near field with FP32 entries, one wave per leaf of at most 64 rows
// (false, with nothing launched, when some leaf holds more)
bool launch_near_leaves(Plan &P, const float *Xs, int NP, double *Y, hipStream_t s);
// the pivot + LU form (lu_form.hip)
constexpr int kLuSlots = 4;                // 64-row register slots of the in-wave solves
constexpr int kLuMaxRank = 64 * kLuSlots;  // largest rank the form takes
constexpr int kLuGroup = 4;                // right-hand sides per pass of its kernels
void lu_pack_batch(Plan &P, const int32_t *list, int64_t q0, int64_t q1, int kws, const double *ws,
                   const int64_t *ws_off, int64_t ws_base, int64_t *scan_buf, hipStream_t s);
void lu_finish(Plan &P, hipStream_t s);
void matvec_lu(Plan &P, const void *x, void *y, int64_t nrhs, int64_t ldx, int64_t ldy,
               int io_dtype, bool adjoint, double *xp, double *yn, double *z, hipStream_t s);
void export_lu(const Plan &P, double *host_out);

// GMRES on (diag I + scale K~) x = f, and the exact dense product (solve.hip)
constexpr int kMaxRestart = 256;
struct SolveResult {
    int iterations = 0, cycles = 0, converged = 0;
    double rel_residual = 0.0;  // true relative residual at exit
    double est_residual = 0.0;  // last Givens estimate
};
SolveResult solve_gmres(Plan &P, double diag, double scale, const double *f, double *x,
                        double rtol, int restart, int max_iter, hipStream_t s);
void dense_matvec(const double *pts, int64_t n, int kind, double kp, const double *x, double *y,
                  hipStream_t s);

// device-wide exclusive scan; out may alias in; returns the total
int64_t scan_exclusive_i64(Plan &P, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
void scan_exclusive_i32_nototal(Plan &P, const int32_t *in, int32_t *out, int64_t n, hipStream_t s);

template <typename T> void to_host(T *dst, const T *src, int64_t n, hipStream_t s) {
    if (n <= 0)
        return;
    H3D_HIP(hipMemcpyAsync(dst, src, sizeof(T) * size_t(n), hipMemcpyDeviceToHost, s));
    H3D_HIP(hipStreamSynchronize(s));
}

inline int grid_for(int64_t n, int block) {
    int64_t g = ceil_div(n, block);
    if (g < 1)
        g = 1;
    return int(g);
}

}  // namespace h3d
