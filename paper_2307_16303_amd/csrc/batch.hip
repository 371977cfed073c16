// Many independent HODLR3D operators multiplied together, phase by phase.
//
// Every problem keeps its own plan (tree, lists, factors: Sec. 2.1, Sec. 4,
// Algorithm 1).  A product of the batch is Algorithm 2 for each problem, cut
// into the same work items as the per-phase kernels use (the gather of 1024
// rows, the near field of one leaf, one stage-1 item, stage 2 of one chunk
// box), and run phase by phase over all problems at once:
//
//   [gather of every problem] [near field of every problem]
//   [stage 1 of every problem and level, one launch per stage-1 shape]
//   [stage 2 of every problem]
//
// (Stage 1 is followed by one launch that adds up the parts of split
// columns.)  Each launch is as large as the sum of the problems' items, so small
// problems fill the GPU together, and each carries only its own kind of work:
// the registers, and so the occupancy, of the per-phase kernels.  The stream
// orders the phases.  A launch's work items are numbered consecutively over a
// run (segment) per problem, or per (problem, level) for stage 1; a wave finds
// its segment by binary search over the segments' first units.  Each member
// keeps its own tuned launch shapes: its stage-1 levels go to the launch of
// their shape, its chunk boxes to the stage-2 launch of its wave count.  The
// arithmetic of each item is the code of the per-phase kernels
// (product_items.hpp), so a member's own product through h3d_matvec gives
// bitwise the same result.  (Members do not fuse the finest level: the batch
// launches do not carry the fused form.)
#include "stage1_items.hpp"

namespace h3d {

enum : int32_t { kSegGather = 0, kSegNear = 1, kSegS1 = 2, kSegS2 = 3, kSegReduce = 4 };

struct BatchSeg {
    int64_t start;  // first unit of the run (units of one launch are consecutive)
    int64_t count;  // items (one per unit) of the run
    int32_t kind, prob, level, shape;
};

struct BatchProb {
    int64_t n;
    int L, lc, kind;
    double kp;
    const int32_t *perm, *leaf_off, *leaf_of, *near_ptr, *near_s;
    const double *px, *py, *pz;
    double *xp, *yn, *z;
    int64_t ldz;
    dev::S2Tab tab;
    const int64_t *grp_begin;
    void *const *uptr;
    const int32_t *rank;
    const int64_t *col0;
    dev::S1Args s1[kMaxLevels + 1];
    // split stage-1 columns of a level: the column groups (first item, parts)
    const int32_t *s1_grp[kMaxLevels + 1];
    int64_t s1_ngrp[kMaxLevels + 1];
};

namespace {

using namespace dev;

constexpr int kGatherRows = 1024;  // rows per gather item
constexpr int kReduceCols = 256;   // split-column sums per reduction item
// workgroups per XCD chunk (xcd_chunks) of the stage-1 and stage-2 launches
constexpr int kS1Chunk = 16, kS2Chunk = 8;

// the stage-1 shapes the batch launches carry: every shape the tuner may
// choose (a split shape runs the wide form's items over parts of columns,
// selected at run time by S1Args::part)
struct ShapeDef {
    int packed, S, U;
};
constexpr ShapeDef kShapes[] = {
    {1, 4, 2},  {1, 4, 4},  {1, 8, 2},  {1, 8, 4},  {1, 16, 2}, {1, 16, 4}, {1, 4, 8},
    {1, 8, 8},  {1, 16, 8}, {0, 8, 4},  {0, 8, 8},  {0, 16, 4}, {0, 16, 8}, {0, 32, 4},
    {0, 32, 8}, {0, 64, 2}, {0, 64, 4}, {0, 64, 8}, {0, 16, 16}, {0, 32, 16}, {0, 64, 16}};
constexpr int kNumS1Shapes = int(sizeof(kShapes) / sizeof(kShapes[0]));
// shapes with twice the loads in flight, built for FP32 / BF16 factors only
constexpr bool narrow_only(int id) {
    return (kShapes[id].packed && kShapes[id].U == 8) || (!kShapes[id].packed && kShapes[id].U == 16);
}

int shape_id(const S1Shape &sh) {
    if (sh.rows > 0 && sh.packed)
        return -1;
    for (int i = 0; i < kNumS1Shapes; ++i)
        if (kShapes[i].packed == sh.packed && kShapes[i].S == sh.S && kShapes[i].U == sh.U)
            return i;
    return -1;
}

// the segment of unit u among segs[sb, se) (their first units ascending);
// u is the same in every lane, and so is the segment, which is read into
// scalar registers
__device__ __forceinline__ BatchSeg seg_of(const BatchSeg *__restrict__ segs, int sb, int se,
                                           int64_t u) {
    int lo = sb, hi = se - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].start <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return segs[__builtin_amdgcn_readfirstlane(lo)];
}

// gather: one workgroup per 1024 rows of a problem
__global__ void __launch_bounds__(256)
    k_bgather(const BatchProb *__restrict__ probs, const BatchSeg *__restrict__ segs, int sb,
              int se, int64_t u0, const void *const *__restrict__ io, int nrhs, int io_f32) {
    const int64_t u = u0 + blockIdx.x;
    const BatchSeg sg = seg_of(segs, sb, se, u);
    const BatchProb &D = probs[sg.prob];
    const int64_t i = u - sg.start;
    const void *x = io[sg.prob];
    for (int r = threadIdx.x; r < kGatherRows; r += 256) {
        const int64_t row = i * kGatherRows + r;
        if (row < D.n)
            gather_row(x, io_f32, D.n, D.n, nrhs, D.perm, D.xp, row);
    }
}

// near field: one wave per leaf
template <int DT>
__global__ void __launch_bounds__(64)
    k_bnear(const BatchProb *__restrict__ probs, const BatchSeg *__restrict__ segs, int sb,
            int se, int64_t u0, int nrhs) {
    const int64_t u = u0 + blockIdx.x;
    const BatchSeg sg = seg_of(segs, sb, se, u);
    const BatchProb &D = probs[sg.prob];
    near_leaf<1, DT != H3D_F64>(u - sg.start, D.leaf_off, D.near_ptr, D.near_s, D.px, D.py,
                                        D.pz, D.kind, D.kp, nrhs, D.xp, D.n, D.yn);
}

// stage 1 of one shape: one work item per wave, four waves per workgroup,
// workgroups renumbered so that every XCD takes a contiguous run of items
template <int DT, int SHAPE>
__global__ void __launch_bounds__(256)
    k_bs1(const BatchProb *__restrict__ probs, const BatchSeg *__restrict__ segs, int sb, int se,
          int64_t u0, int64_t units) {
    const int64_t b = xcd_chunks<kS1Chunk>(blockIdx.x, gridDim.x);
    const int64_t w = uniform64((b * blockDim.x + threadIdx.x) >> 6);
    if (w >= units)
        return;
    const BatchSeg sg = seg_of(segs, sb, se, u0 + w);
    // the level's arguments, read once with scalar loads; the item code reads
    // through their pointers with global (not flat) instructions (glob), which
    // gives this kernel the registers of the single-problem k_s1_wide and
    // k_s1_packed
    const S1Args a = probs[sg.prob].s1[sg.level];
    const int64_t i = u0 + w - sg.start;
    constexpr ShapeDef sh = kShapes[SHAPE];
    if constexpr (sh.packed)
        s1_packed_item<sh.S, sh.U, DT, 1>(a, i);
    else
        s1_wide_item<sh.S, sh.U, DT, 1>(a, i);
}

// split stage-1 columns of one (problem, level): kReduceCols sums per item
__global__ void __launch_bounds__(kReduceCols)
    k_bs1_reduce(const BatchProb *__restrict__ probs, const BatchSeg *__restrict__ segs, int sb,
                 int se, int64_t u0) {
    const int64_t u = u0 + blockIdx.x;
    const BatchSeg sg = seg_of(segs, sb, se, u);
    const BatchProb &D = probs[sg.prob];
    s1_reduce_column((u - sg.start) * kReduceCols + threadIdx.x, D.s1_ngrp[sg.level],
                     D.s1_grp[sg.level], D.s1[sg.level]);
}

// stage 2: one workgroup of W waves per chunk box, written straight to y
// (FP64 factors, one RHS: four waves per SIMD, as k_stage2)
template <int DT, int W>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(DT == H3D_F64 ? 4 : 1)))
    k_bs2(const BatchProb *__restrict__ probs, const BatchSeg *__restrict__ segs, int sb, int se,
          int64_t u0, int nprob, const void *const *__restrict__ io, int nrhs, int io_f32) {
    const int64_t u = u0 + xcd_chunks<kS2Chunk>(blockIdx.x, gridDim.x);
    const BatchSeg sg = seg_of(segs, sb, se, u);
    const BatchProb &D = probs[sg.prob];
    stage2_chunk<DT, 1, W>(u - sg.start, D.tab, D.leaf_off, D.leaf_of, D.grp_begin, nullptr,
                           D.uptr, D.rank, D.col0, D.z, D.ldz, D.yn, D.n, nrhs, D.perm,
                           const_cast<void *>(io[nprob + sg.prob]), D.n, io_f32, 1, D.L, nullptr);
}

// Before each product: the x and y pointers of up to kIoPerLaunch problems
// into the device table.
constexpr int kIoPerLaunch = 32;
struct IoChunk {
    const void *x[kIoPerLaunch];
    void *y[kIoPerLaunch];
};

__global__ void k_batch_prepare(IoChunk c, int base, int count, int nprob, const void **io) {
    const int t = threadIdx.x;
    if (t < count) {
        io[base + t] = c.x[t];
        io[nprob + base + t] = c.y[t];
    }
}

// one launch of the batch: segments [sb, se), units [u0, u0 + units)
enum : int { kLaunchKind, kLaunchShape, kLaunchSb, kLaunchSe, kLaunchU0, kLaunchUnits, kLaunchLen };

}  // namespace

// Builds the segments (one unit per work item), grouped by launch: gather,
// near field, stage 1 by shape, the sums of split columns, stage 2 by waves
// per chunk box; one list of
// launches for one right-hand side (the members' tuned shapes) and one for
// two to seven (their shapes for several right-hand sides).
void batch_setup(h3d_plan &bp, hipStream_t s) {
    BatchState &B = *bp.batch;
    Plan &P = bp.P;
    const int nprob = int(B.subs.size());
    std::vector<BatchSeg> segs;
    int64_t pos = 0;
    auto add = [&](int32_t kind, int32_t prob, int32_t level, int32_t shape, int64_t count) {
        if (count > 0) {
            segs.push_back(BatchSeg{pos, count, kind, prob, level, shape});
            pos += count;
        }
    };
    for (int cls = 0; cls < 2; ++cls) {
        std::vector<int64_t> &Ls = B.launches[cls];
        Ls.clear();
        // one launch over the segments added by `body`
        auto launch = [&](int kind, int shape, auto body) {
            const int sb = int(segs.size());
            const int64_t u0 = pos;
            body();
            if (int(segs.size()) > sb)
                Ls.insert(Ls.end(), {int64_t(kind), int64_t(shape), int64_t(sb),
                                     int64_t(segs.size()), u0, pos - u0});
        };
        launch(kSegGather, 0, [&] {
            for (int p = 0; p < nprob; ++p)
                add(kSegGather, p, 0, 0, ceil_div(B.subs[size_t(p)]->P.n, kGatherRows));
        });
        launch(kSegNear, 0, [&] {
            for (int p = 0; p < nprob; ++p)
                add(kSegNear, p, 0, 0, pow8(B.subs[size_t(p)]->P.L));
        });
        for (int p = 0; p < nprob; ++p) {
            const Plan &Q = B.subs[size_t(p)]->P;
            for (int l = 1; l <= Q.L; ++l)
                if (Q.s1_nitems[cls][l] > 0 && shape_id(Q.s1_shape[cls][l]) < 0)
                    fail(H3D_EDEVICE, "internal: stage-1 shape not carried by the batch kernels");
        }
        for (int sh = 0; sh < kNumS1Shapes; ++sh)
            launch(kSegS1, sh, [&] {
                for (int p = 0; p < nprob; ++p) {
                    const Plan &Q = B.subs[size_t(p)]->P;
                    for (int l = 1; l <= Q.L; ++l)
                        if (Q.s1_nitems[cls][l] > 0 && shape_id(Q.s1_shape[cls][l]) == sh)
                            add(kSegS1, p, l, sh, Q.s1_nitems[cls][l]);
                }
            });
        // split columns (one right-hand side only), once every stage-1 launch
        // has written its partial sums
        launch(kSegReduce, 0, [&] {
            for (int p = 0; p < nprob; ++p) {
                const Plan &Q = B.subs[size_t(p)]->P;
                for (int l = 1; l <= Q.L; ++l)
                    if (cls == 0 && Q.s1_nitems[0][l] > 0 && Q.s1_part[l])
                        add(kSegReduce, p, l, 0,
                            ceil_div(Q.s1_ngrp[l] * Q.s1_span[0][l], int64_t(kReduceCols)));
            }
        });
        for (int w : {1, 2, 4, 8})
            launch(kSegS2, w, [&] {
                for (int p = 0; p < nprob; ++p) {
                    const Plan &Q = B.subs[size_t(p)]->P;
                    const int qw = Q.s2_waves[cls];
                    if ((qw <= 1 ? 1 : qw <= 2 ? 2 : qw <= 4 ? 4 : 8) == w)
                        add(kSegS2, p, 0, w, pow8(Q.chunk_level));
                }
            });
    }
    B.nseg = int(segs.size());
    B.nitems = pos;
    if (pos >= int64_t(0x7fffffff))
        fail(H3D_EINVAL, "batch too large: more than 2^31 work items");
    B.segs = static_cast<BatchSeg *>(P.mem.alloc(sizeof(BatchSeg) * std::max<size_t>(segs.size(), 1)));
    if (!segs.empty())
        H3D_HIP(hipMemcpy(B.segs, segs.data(), sizeof(BatchSeg) * segs.size(),
                          hipMemcpyHostToDevice));
    B.probs = static_cast<BatchProb *>(P.mem.alloc(sizeof(BatchProb) * size_t(nprob)));
    B.io = static_cast<const void **>(P.mem.alloc(sizeof(void *) * 2 * size_t(nprob)));
    (void)s;
}

// Writes the per-problem descriptors for nrhs right-hand sides.
static void write_descriptors(BatchState &B, int64_t nrhs) {
    const int cls = nrhs == 1 ? 0 : 1;
    const int nprob = int(B.subs.size());
    std::vector<BatchProb> d(static_cast<size_t>(nprob));
    std::vector<const void *> scr;
    for (int p = 0; p < nprob; ++p) {
        Plan &Q = B.subs[size_t(p)]->P;
        BatchProb &D = d[size_t(p)];
        std::memset(&D, 0, sizeof(D));
        D.n = Q.n;
        D.L = Q.L;
        D.lc = Q.chunk_level;
        D.kind = Q.cfg.kernel;
        D.kp = Q.cfg.kernel_param;
        D.perm = Q.perm;
        D.leaf_off = Q.leaf_off;
        D.leaf_of = Q.leaf_of;
        D.near_ptr = Q.near_ptr;
        D.near_s = Q.near_s;
        D.px = Q.px;
        D.py = Q.py;
        D.pz = Q.pz;
        D.xp = Q.xp;
        D.yn = Q.yp;
        D.z = Q.z;
        D.ldz = Q.ncols;
        for (int l = 0; l <= kMaxLevels; ++l)
            D.tab.box_base[l] = Q.box_base[l];
        D.tab.L = Q.L;
        D.tab.lc = Q.chunk_level;
        D.tab.panel = 1;
        D.grp_begin = Q.tgt_begin;
        D.uptr = Q.blk_uptr;
        D.rank = Q.blk_rank;
        D.col0 = Q.blk_col0;
        for (int l = 1; l <= Q.L; ++l) {
            S1Args &a = D.s1[l];
            a.items = reinterpret_cast<const int2 *>(Q.s1_items[cls][l]);
            a.nitems = Q.s1_nitems[cls][l];
            a.span = Q.s1_span[cls][l];
            a.blk_col0 = Q.blk_col0;
            a.rank = Q.blk_rank;
            a.seg_len = Q.blk_n;
            a.seg_off = Q.blk_soff;
            a.seg_ptr = Q.blk_vptr;
            a.scale2 = Q.blk_scale;
            a.nrhs = int(nrhs);
            a.xp = Q.xp;
            a.n = Q.n;
            a.z = Q.z;
            a.ldz = Q.ncols;
            // split columns, as the member's own stage 1 (stage1_args)
            if (cls == 0 && Q.s1_part[l]) {
                a.part = Q.s1_part[l];
                a.rows = Q.s1_shape[0][l].rows;
                a.zp = Q.s1_zp[l];
                D.s1_grp[l] = Q.s1_grp[l];
                D.s1_ngrp[l] = Q.s1_ngrp[l];
            }
        }
        scr.push_back(Q.xp);
        scr.push_back(Q.yp);
        scr.push_back(Q.z);
    }
    H3D_HIP(hipMemcpy(B.probs, d.data(), sizeof(BatchProb) * d.size(), hipMemcpyHostToDevice));
    B.desc_nrhs = nrhs;
    B.desc_scratch = scr;
}

// stage 1 of shape `id` (a compile-time constant from a run-time index)
template <int DT, int ID = 0>
static void launch_bs1(int id, int g, const BatchState &B, int sb, int se, int64_t u0,
                       int64_t units, hipStream_t s) {
    if constexpr (ID < kNumS1Shapes) {
        if (id != ID) {
            launch_bs1<DT, ID + 1>(id, g, B, sb, se, u0, units, s);
        } else if constexpr (DT == H3D_F64 && narrow_only(ID)) {
            fail(H3D_EDEVICE, "internal: a narrow-factor stage-1 shape on FP64 factors");
        } else {
            k_bs1<DT, ID><<<g, 256, 0, s>>>(B.probs, B.segs, sb, se, u0, units);
        }
    } else {
        fail(H3D_EDEVICE, "internal: unknown stage-1 shape of a batch launch");
    }
}

// the phase launches of one product, in order
template <int DT>
static void batch_launches(const BatchState &B, int nprob, int nrhs, int io_f32, hipStream_t s) {
    const std::vector<int64_t> &Ls = B.launches[nrhs == 1 ? 0 : 1];
    for (size_t j = 0; j + kLaunchLen <= Ls.size(); j += kLaunchLen) {
        const int64_t *L = Ls.data() + j;
        const int kind = int(L[kLaunchKind]), shape = int(L[kLaunchShape]);
        const int sb = int(L[kLaunchSb]), se = int(L[kLaunchSe]);
        const int64_t u0 = L[kLaunchU0], units = L[kLaunchUnits];
        switch (kind) {
        case kSegGather:
            k_bgather<<<int(units), 256, 0, s>>>(B.probs, B.segs, sb, se, u0, B.io, nrhs, io_f32);
            break;
        case kSegNear:
            k_bnear<DT><<<int(units), 64, 0, s>>>(B.probs, B.segs, sb, se, u0, nrhs);
            break;
        case kSegS1:
            launch_bs1<DT>(shape, int((units + 3) / 4), B, sb, se, u0, units, s);
            break;
        case kSegReduce:
            k_bs1_reduce<<<int(units), kReduceCols, 0, s>>>(B.probs, B.segs, sb, se, u0);
            break;
        default:
#define H3D_BS2(W)                                                                              \
    k_bs2<DT, W><<<int(units), 64 * W, 0, s>>>(B.probs, B.segs, sb, se, u0, nprob, B.io, nrhs,   \
                                               io_f32)
            if (shape == 1)
                H3D_BS2(1);
            else if (shape == 2)
                H3D_BS2(2);
            else if (shape == 4)
                H3D_BS2(4);
            else
                H3D_BS2(8);
#undef H3D_BS2
            break;
        }
        H3D_LAUNCH_CHECK();
    }
}

void batch_run(h3d_plan &bp, const void *const *x, void *const *y, int64_t nrhs, int io_dtype,
               hipStream_t s) {
    BatchState &B = *bp.batch;
    Plan &P = bp.P;
    const int nprob = int(B.subs.size());
    if (nrhs >= kBatchedMinRhs) {
        // Eight or more right-hand sides: every problem's product is a set of
        // dense GEMMs on the matrix cores, large enough to fill the GPU on its
        // own, so the problems run back to back on the stream.
        hipEvent_t ev = P.prof.begin(s);
        double bytes = 0.0, flops = 0.0;
        for (int p = 0; p < nprob; ++p) {
            Plan &Q = B.subs[size_t(p)]->P;
            matvec_batched(Q, x[p], y[p], nrhs, Q.n, Q.n, io_dtype, false, s);
            bytes += double(Q.stats.factor_bytes);
            flops += 2.0 * double(Q.stats.factor_entries) * double(nrhs);
        }
        P.prof.end(s, ev, "k_batch_mfma", bytes, flops);
        return;
    }
    bool fresh = B.desc_nrhs != nrhs;
    for (int p = 0; p < nprob; ++p) {
        Plan &Q = B.subs[size_t(p)]->P;
        ensure_scratch(Q, nrhs, s);
        const size_t k = 3 * size_t(p);
        if (B.desc_scratch.size() != 3 * size_t(nprob) || B.desc_scratch[k] != Q.xp ||
            B.desc_scratch[k + 1] != Q.yp || B.desc_scratch[k + 2] != Q.z)
            fresh = true;
    }
    if (fresh) {
        // the descriptors sit in device memory that captured graphs of the
        // batch read at every replay
        if (P.live_graphs > 0)
            fail(H3D_EINVAL, "a batch product with other right-hand sides would rewrite the "
                             "problem descriptors that captured graphs of the batch use: "
                             "destroy them first");
        H3D_HIP(hipStreamSynchronize(s));
        write_descriptors(B, nrhs);
    }
    for (int base = 0; base < nprob; base += kIoPerLaunch) {
        IoChunk c{};
        const int cnt = std::min(kIoPerLaunch, nprob - base);
        for (int j = 0; j < cnt; ++j) {
            c.x[j] = x[base + j];
            c.y[j] = y[base + j];
        }
        k_batch_prepare<<<1, 64, 0, s>>>(c, base, cnt, nprob, B.io);
        H3D_LAUNCH_CHECK();
    }
    const int io_f32 = io_dtype == H3D_F32;
    double bytes = 0.0, flops = 0.0;
    for (h3d_plan *q : B.subs) {
        const Plan &Q = q->P;
        bytes += double(Q.stats.factor_bytes) +
                 double(Q.n) * ((io_f32 ? 8.0 : 16.0) + 4.0) * double(nrhs);
        flops += 2.0 * double(Q.stats.factor_entries) * double(nrhs);
    }
    hipEvent_t ev = P.prof.begin(s);
    switch (P.factor_dtype) {
    case H3D_F64:
        batch_launches<H3D_F64>(B, nprob, int(nrhs), io_f32, s);
        break;
    case H3D_F32:
        batch_launches<H3D_F32>(B, nprob, int(nrhs), io_f32, s);
        break;
    default:
        batch_launches<H3D_BF16_SCALED>(B, nprob, int(nrhs), io_f32, s);
        break;
    }
    P.prof.end(s, ev, "k_batch", bytes, flops);
}

// The phase launches have no waits between problems: nothing can give up.
bool batch_wait_failed(h3d_plan &bp, hipStream_t s) {
    (void)bp;
    H3D_HIP(hipStreamSynchronize(s));
    return false;
}

}  // namespace h3d
