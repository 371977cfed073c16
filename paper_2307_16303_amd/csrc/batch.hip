// Many independent HODLR3D operators multiplied in one persistent launch.
//
// Every problem keeps its own plan (tree, lists, factors: Sec. 2.1, Sec. 4,
// Algorithm 1).  A product of the batch is Algorithm 2 for each problem, cut
// into the same work items as the per-phase kernels use (the gather of 1024
// rows, the near field of one leaf, one stage-1 item, stage 2 of one chunk
// box) and put in one queue:
//
//   [gather of every problem] [near + stage 1 of problem 0] [... of problem 1]
//   ... [stage 2 of every problem]
//
// The queue is cut into units: a run of consecutive items of one kind and
// problem, sized so that a unit streams about kUnitBytes of factors (one
// chunk box for stage 2, 64 leaves for the near field).  One-wave
// workgroups, as many as are resident at once, take units in order from a
// global ticket counter; per unit a wave issues one ticket atomic, one
// release fence and one counter increment.  Two counters per problem order
// the phases: near-field and stage-1 units wait until the problem's gather
// units are done, stage-2 units until its near-field and stage-1 units are
// done.  Units are taken in queue order and every wait is for units earlier
// in the queue, which running waves already hold, so every wait ends; the waits are bounded nevertheless, and a wave that gives up
// sets an error flag (h3d_batch_check) and carries on, so the launch always
// drains.  The arithmetic of each item is the code of the per-phase kernels
// (product_items.hpp) with one wave per stage-2 chunk box: a problem's plan
// configured that way (the batch sets it so) gives bitwise the same product
// through h3d_matvec.
#include "stage1_items.hpp"

namespace h3d {

enum : int32_t { kSegGather = 0, kSegNear = 1, kSegS1 = 2, kSegS2 = 3 };

struct BatchSeg {
    int64_t start;     // first queue unit of the run
    int64_t count;     // items of the run
    int32_t per_unit;  // items per unit
    int32_t kind, prob, level, shape;
};

struct BatchProb {
    int64_t n;
    int L, lc, kind;
    double kp;
    unsigned n_gather;  // units before near field and stage 1 may start
    unsigned n_mid;     // near-field and stage-1 units before stage 2 may start
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
};

namespace {

using namespace dev;

constexpr int kGatherRows = 1024;           // rows per gather item
constexpr int kNearPerUnit = 64;            // leaves per near-field unit
constexpr double kUnitBytes = 1 << 20;      // factor bytes per stage-1 unit
constexpr int64_t kSpinLimit = int64_t(1) << 20;  // polls: about a second

// stage-1 shapes the persistent kernel carries (the default shapes)
int shape_id(const S1Shape &sh) {
    if (sh.rows > 0)
        return -1;
    if (sh.packed && sh.S == 4 && sh.U == 4)
        return 0;
    if (sh.packed && sh.S == 8 && sh.U == 4)
        return 1;
    if (!sh.packed && sh.S == 16 && sh.U == 4)
        return 2;
    if (!sh.packed && sh.S == 64 && sh.U == 8)
        return 3;
    if (!sh.packed && sh.S == 64 && sh.U == 4)
        return 4;
    return -1;
}

// lane 0 polls until *cnt reaches target (bounded), then the wave acquires
__device__ __forceinline__ void wait_for(unsigned *cnt, unsigned target, unsigned *err) {
    if (threadIdx.x == 0) {
        int64_t polls = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++polls > kSpinLimit) {
                __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// the wave's writes become visible, then the unit is counted
__device__ __forceinline__ void unit_done(unsigned *cnt) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DT>
__global__ void __launch_bounds__(64)
    k_batch(const BatchProb *__restrict__ probs, const BatchSeg *__restrict__ segs, int nseg,
            int64_t nunits, unsigned *ctl, int nprob, const void *const *__restrict__ io,
            int nrhs, int io_f32) {
    const int lane = threadIdx.x;
    unsigned *head = ctl, *err = ctl + 1, *done_g = ctl + 2, *done_m = ctl + 2 + nprob;
    int acq_g = -1, acq_m = -1;  // last problem whose inputs this wave has acquired
    for (;;) {
        unsigned tk = 0;
        if (lane == 0)
            tk = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t u = int64_t(uint32_t(__builtin_amdgcn_readfirstlane(__shfl(tk, 0))));
        if (u >= nunits)
            return;
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].start <= u)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchSeg &sg = segs[lo];
        const int kind = sg.kind, p = sg.prob;
        const int64_t i0 = (u - sg.start) * sg.per_unit;
        const int64_t i1 = min(i0 + sg.per_unit, sg.count);
        const BatchProb &D = probs[p];
        if (kind == kSegGather) {
            const void *x = io[p];
            for (int64_t i = i0; i < i1; ++i)
                for (int r = lane; r < kGatherRows; r += 64) {
                    const int64_t row = i * kGatherRows + r;
                    if (row < D.n)
                        gather_row(x, io_f32, D.n, D.n, nrhs, D.perm, D.xp, row);
                }
            unit_done(done_g + p);
        } else if (kind == kSegS2) {
            if (acq_m != p) {
                wait_for(done_m + p, D.n_mid, err);
                acq_m = p;
            }
            for (int64_t i = i0; i < i1; ++i)
                stage2_chunk<DT, 1, 1, true>(i, D.tab, D.leaf_off, D.leaf_of, D.grp_begin, nullptr,
                                             D.uptr, D.rank, D.col0, D.z, D.ldz, D.yn, D.n, nrhs,
                                             D.perm, const_cast<void *>(io[nprob + p]), D.n,
                                             io_f32, 1, D.L, nullptr);
        } else {
            if (acq_g != p) {
                wait_for(done_g + p, D.n_gather, err);
                acq_g = p;
            }
            if (kind == kSegNear) {
                for (int64_t i = i0; i < i1; ++i)
                    near_leaf<1, true, DT != H3D_F64>(i, D.leaf_off, D.near_ptr, D.near_s, D.px,
                                                      D.py, D.pz, D.kind, D.kp, nrhs, D.xp,
                                                      D.n, D.yn);
            } else {
                const S1Args &a = D.s1[sg.level];
                switch (sg.shape) {
                case 0:
                    for (int64_t i = i0; i < i1; ++i)
                        s1_packed_item<4, 4, DT, 1, true>(a, i);
                    break;
                case 1:
                    for (int64_t i = i0; i < i1; ++i)
                        s1_packed_item<8, 4, DT, 1, true>(a, i);
                    break;
                case 2:
                    for (int64_t i = i0; i < i1; ++i)
                        s1_wide_item<16, 4, DT, 1, true>(a, i);
                    break;
                case 3:
                    for (int64_t i = i0; i < i1; ++i)
                        s1_wide_item<64, 8, DT, 1, true>(a, i);
                    break;
                default:
                    for (int64_t i = i0; i < i1; ++i)
                        s1_wide_item<64, 4, DT, 1, true>(a, i);
                    break;
                }
            }
            unit_done(done_m + p);
        }
    }
}

// Before each product: the x and y pointers of up to kIoPerLaunch problems
// into the device table, and (first launch) the queue head, the error flag
// and the per-problem counters set to zero.
constexpr int kIoPerLaunch = 32;
struct IoChunk {
    const void *x[kIoPerLaunch];
    void *y[kIoPerLaunch];
};

__global__ void k_batch_prepare(IoChunk c, int base, int count, int nprob, const void **io,
                                unsigned *ctl, int nctl) {
    const int t = threadIdx.x;
    if (t < count) {
        io[base + t] = c.x[t];
        io[nprob + base + t] = c.y[t];
    }
    if (base == 0)
        for (int j = t; j < nctl; j += blockDim.x)
            ctl[j] = 0u;
}

template <int DT> int resident_grid() {
    int dev = 0, cus = 0, per_cu = 0;
    H3D_HIP(hipGetDevice(&dev));
    H3D_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    H3D_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<DT>, 64, 0));
    return std::max(1, cus) * std::max(1, per_cu);
}

}  // namespace

// Builds the queue (segments and per-problem counts) and the control arrays.
void batch_setup(h3d_plan &bp, hipStream_t s) {
    BatchState &B = *bp.batch;
    Plan &P = bp.P;
    const int nprob = int(B.subs.size());
    const double es = P.factor_dtype == H3D_F64 ? 8.0 : (P.factor_dtype == H3D_F32 ? 4.0 : 2.0);
    std::vector<BatchSeg> segs;
    int64_t pos = 0;
    auto add = [&](int32_t kind, int32_t prob, int32_t level, int32_t shape, int64_t count,
                   int64_t per_unit) {
        if (count <= 0)
            return int64_t(0);
        per_unit = std::max<int64_t>(1, std::min<int64_t>(per_unit, 1 << 20));
        const int64_t units = ceil_div(count, per_unit);
        segs.push_back(BatchSeg{pos, count, int32_t(per_unit), kind, prob, level, shape});
        pos += units;
        return units;
    };
    B.n_gather.assign(size_t(nprob), 0);
    B.n_mid.assign(size_t(nprob), 0);
    for (int p = 0; p < nprob; ++p)
        B.n_gather[size_t(p)] =
            add(kSegGather, p, 0, 0, ceil_div(B.subs[size_t(p)]->P.n, kGatherRows), 1);
    for (int p = 0; p < nprob; ++p) {
        Plan &Q = B.subs[size_t(p)]->P;
        int64_t mid = add(kSegNear, p, 0, 0, pow8(Q.L), kNearPerUnit);
        for (int l = 1; l <= Q.L; ++l) {
            const int64_t ni = Q.s1_nitems[0][l];
            if (ni == 0)
                continue;
            const int id = shape_id(Q.s1_shape[0][l]);
            if (id < 0)
                fail(H3D_EDEVICE, "internal: stage-1 shape not carried by the batch kernel");
            const double item_bytes = double(Q.lvl_entries_v[l]) * es / double(ni);
            mid += add(kSegS1, p, l, id, ni, int64_t(kUnitBytes / std::max(item_bytes, 1.0)));
        }
        B.n_mid[size_t(p)] = mid;
    }
    for (int p = 0; p < nprob; ++p)
        add(kSegS2, p, 0, 0, pow8(B.subs[size_t(p)]->P.chunk_level), 1);
    B.nseg = int(segs.size());
    B.nitems = pos;
    if (pos >= int64_t(0x7fffffff) - (int64_t(1) << 24))
        fail(H3D_EINVAL, "batch queue too long");
    B.segs = static_cast<BatchSeg *>(P.mem.alloc(sizeof(BatchSeg) * segs.size()));
    H3D_HIP(hipMemcpy(B.segs, segs.data(), sizeof(BatchSeg) * segs.size(), hipMemcpyHostToDevice));
    B.probs = static_cast<BatchProb *>(P.mem.alloc(sizeof(BatchProb) * size_t(nprob)));
    B.ctl = P.mem.alloc_n<unsigned>(2 + 2 * int64_t(nprob));
    B.io = static_cast<const void **>(P.mem.alloc(sizeof(void *) * 2 * size_t(nprob)));
    int g = 0;
    switch (P.factor_dtype) {
    case H3D_F64:
        g = resident_grid<H3D_F64>();
        break;
    case H3D_F32:
        g = resident_grid<H3D_F32>();
        break;
    default:
        g = resident_grid<H3D_BF16_SCALED>();
        break;
    }
    B.grid = int(std::min<int64_t>(g, pos));
    (void)s;
}

// Writes the per-problem descriptors for nrhs right-hand sides.
static void write_descriptors(BatchState &B, int64_t nrhs) {
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
        D.n_gather = unsigned(B.n_gather[size_t(p)]);
        D.n_mid = unsigned(B.n_mid[size_t(p)]);
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
            a.items = reinterpret_cast<const int2 *>(Q.s1_items[0][l]);
            a.nitems = Q.s1_nitems[0][l];
            a.span = Q.s1_span[0][l];
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
        }
        scr.push_back(Q.xp);
        scr.push_back(Q.yp);
        scr.push_back(Q.z);
    }
    H3D_HIP(hipMemcpy(B.probs, d.data(), sizeof(BatchProb) * d.size(), hipMemcpyHostToDevice));
    B.desc_nrhs = nrhs;
    B.desc_scratch = scr;
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
    const int nctl = 2 + 2 * nprob;
    for (int base = 0; base < nprob; base += kIoPerLaunch) {
        IoChunk c{};
        const int cnt = std::min(kIoPerLaunch, nprob - base);
        for (int j = 0; j < cnt; ++j) {
            c.x[j] = x[base + j];
            c.y[j] = y[base + j];
        }
        k_batch_prepare<<<1, 256, 0, s>>>(c, base, cnt, nprob, B.io, B.ctl, nctl);
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
        k_batch<H3D_F64><<<B.grid, 64, 0, s>>>(B.probs, B.segs, B.nseg, B.nitems, B.ctl, nprob,
                                                B.io, int(nrhs), io_f32);
        break;
    case H3D_F32:
        k_batch<H3D_F32><<<B.grid, 64, 0, s>>>(B.probs, B.segs, B.nseg, B.nitems, B.ctl, nprob,
                                                B.io, int(nrhs), io_f32);
        break;
    default:
        k_batch<H3D_BF16_SCALED><<<B.grid, 64, 0, s>>>(B.probs, B.segs, B.nseg, B.nitems, B.ctl,
                                                        nprob, B.io, int(nrhs), io_f32);
        break;
    }
    H3D_LAUNCH_CHECK();
    P.prof.end(s, ev, "k_batch", bytes, flops);
}

// Synchronises s and reports whether a wait of the last products gave up.
bool batch_wait_failed(h3d_plan &bp, hipStream_t s) {
    BatchState &B = *bp.batch;
    unsigned flag = 0;
    H3D_HIP(hipMemcpyAsync(&flag, B.ctl + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    H3D_HIP(hipStreamSynchronize(s));
    return flag != 0;
}

}  // namespace h3d
