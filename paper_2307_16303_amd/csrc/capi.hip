// C ABI of libhodlr3d (declared in include/hodlr3d.h): argument validation,
// plan lifecycle, statistics, export and profiling.  No exception crosses the
// ABI; failures return an h3d_status and leave a message for h3d_last_error.
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>

#include "h3d_internal.hpp"

h3d_plan::~h3d_plan() { delete batch; }

struct h3d_graph {
    h3d_plan *plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool batch = false;  // a batch product: the members' scratch is pinned too
};

namespace h3d {
void near_pair_count(Plan &P, hipStream_t s);
bool batch_wait_failed(h3d_plan &bp, hipStream_t s);
}

namespace {

thread_local std::string g_last_error;

// Handles the library has handed out and not yet released.  Every entry point
// looks its handle up here first, so a destroyed (or never created) handle
// gives an error instead of a use of freed memory.
enum HandleKind { kOwnPlan = 1, kMemberPlan = 2, kGraph = 3 };
std::mutex g_reg_mu;
std::unordered_map<const void *, int> g_reg;

void reg_add(const void *h, int kind) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_reg[h] = kind;
}
void reg_del(const void *h) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_reg.erase(h);
}
int reg_kind(const void *h) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_reg.find(h);
    return it == g_reg.end() ? 0 : it->second;
}

// H3D_OK for a live, built plan (own or batch member); H3D_ENOTBUILT otherwise.
h3d_status plan_status(const h3d_plan *plan) {
    if (!plan)
        return g_last_error = "plan is NULL", H3D_ENOTBUILT;
    const int k = reg_kind(plan);
    if (k != kOwnPlan && k != kMemberPlan)
        return g_last_error = "not a live plan (destroyed, or never returned by a build call)",
               H3D_ENOTBUILT;
    if (!plan->P.built)
        return g_last_error = "plan is not built", H3D_ENOTBUILT;
    return H3D_OK;
}

template <class F> h3d_status guarded(F &&f) {
    try {
        f();
        return H3D_OK;
    } catch (const h3d::Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return H3D_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return H3D_EDEVICE;
    } catch (...) {
        g_last_error = "unknown failure";
        return H3D_EDEVICE;
    }
}

h3d_status invalid(const std::string &m) {
    g_last_error = m;
    return H3D_EINVAL;
}

// Runs f with the plan's device current, restoring the caller's device.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev)
            H3D_HIP(hipSetDevice(dev));
        else
            prev = -1;
    }
    ~DeviceScope() {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

size_t io_size(int32_t dt) { return dt == H3D_F32 ? 4 : 8; }

h3d_status batch_plan_error() {
    return invalid("a batch plan takes h3d_matvec_batch; h3d_batch_plan gives its problems");
}

h3d_status matvec_check(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                        int64_t ldy, int32_t io) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    if (plan->batch)
        return batch_plan_error();
    h3d::Plan &P = plan->P;
    if (!x || !y)
        return invalid("x and y must be device pointers");
    if (nrhs < 1)
        return invalid("nrhs must be >= 1");
    if (ldx < P.n || ldy < P.n)
        return invalid("leading dimensions must be >= n");
    if (io != H3D_F64 && io != H3D_F32)
        return invalid("io_dtype must be H3D_F64 or H3D_F32");
    const size_t es = io_size(io);
    const uintptr_t xa = uintptr_t(x), xb = xa + size_t((nrhs - 1) * ldx + P.n) * es;
    const uintptr_t ya = uintptr_t(y), yb = ya + size_t((nrhs - 1) * ldy + P.n) * es;
    if (xa < yb && ya < xb)
        return invalid("x and y overlap");
    return H3D_OK;
}

h3d_status matvec_common(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                         int64_t ldy, int32_t io, void *stream, bool adjoint) {
    const h3d_status st = matvec_check(plan, x, y, nrhs, ldx, ldy, io);
    if (st != H3D_OK)
        return st;
    h3d::Plan &P = plan->P;
    return guarded([&] {
        DeviceScope ds(P.device);
        h3d::matvec_run(P, x, y, nrhs, ldx, ldy, io, adjoint, static_cast<hipStream_t>(stream));
    });
}

h3d_status check_config(const h3d_config *cfg, const h3d_allocator *alloc) {
    if (!cfg)
        return invalid("cfg must not be NULL");
    if (cfg->kernel < H3D_LAPLACE || cfg->kernel > H3D_COS_R)
        return invalid("unknown kernel");
    if (!std::isfinite(cfg->kernel_param))
        return invalid("kernel_param must be finite");
    if (cfg->leaf_size < 1)
        return invalid("leaf_size must be >= 1");
    if (!(cfg->tol > 0.0 && cfg->tol < 1.0))
        return invalid("tol must lie in (0, 1)");
    if (cfg->factor_dtype < H3D_F64 || cfg->factor_dtype > H3D_BF16_SCALED)
        return invalid("unknown factor_dtype");
    if (cfg->max_depth < 0 || cfg->max_depth > h3d::kMaxDepth)
        return invalid("max_depth must lie in [0, 10]");
    if (!std::isfinite(cfg->box_side))
        return invalid("box_side must be finite");
    if (cfg->box_side > 0.0)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(cfg->box_lo[a]))
                return invalid("box_lo must be finite");
    if (alloc && ((alloc->alloc == nullptr) != (alloc->free == nullptr)))
        return invalid("allocator needs both alloc and free");
    if ((cfg->flags & H3D_FLAG_TRUNCATE) && (cfg->flags & H3D_FLAG_KEEP_PIVOTS))
        return invalid("truncated factors have no ACA pivots: H3D_FLAG_TRUNCATE excludes "
                       "H3D_FLAG_KEEP_PIVOTS");
    if (cfg->flags & H3D_FLAG_LU_FORM) {
        if (cfg->flags & H3D_FLAG_TRUNCATE)
            return invalid("the pivot + LU form keeps the ACA pivots: H3D_FLAG_LU_FORM excludes "
                           "H3D_FLAG_TRUNCATE");
        if (cfg->factor_dtype != H3D_F64)
            return invalid("the pivot + LU form stores FP64 LU factors: factor_dtype must be "
                           "H3D_F64");
    }
    return H3D_OK;
}

// Builds one operator (throws h3d::Error).  A member of a batch is tuned as
// well, among the forms the batch launches carry (every stage-1 shape; the
// finest level not fused).
h3d_plan *build_plan(const double *points, int64_t n, const h3d_config &cfg,
                     const h3d_allocator *alloc, hipStream_t s, bool in_batch) {
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<h3d_plan> plan(new h3d_plan());
    h3d::Plan &P = plan->P;
    P.cfg = cfg;
    H3D_HIP(hipGetDevice(&P.device));
    P.mem.configure(alloc, s);
    P.n = n;
    P.in_batch = in_batch;
    try {
        h3d::tree_build(P, points, s);
        h3d::lists_build(P, s);
        h3d::factors_build(P, s);
        h3d::near_pair_count(P, s);
        if (!(P.cfg.flags & H3D_FLAG_NO_AUTOTUNE))
            h3d::autotune(P, 1, s);
    } catch (...) {
        // kernels queued before the failure finish before the plan's memory
        // goes back to the allocator
        (void)hipStreamSynchronize(s);
        throw;
    }
    H3D_HIP(hipStreamSynchronize(s));
    h3d_stats &S = P.stats;
    S.n = n;
    S.depth = P.L;
    S.factor_dtype = P.factor_dtype;
    for (int a = 0; a < 3; ++a)
        S.box_lo[a] = P.lo[a];
    S.box_side = P.side;
    S.n_far = P.nfar;
    S.n_near = P.nnear;
    for (int l = 0; l < H3D_MAX_LEVELS; ++l)
        S.far_per_level[l] = (l >= 1 && l <= P.L) ? P.lvl_blk[l + 1] - P.lvl_blk[l] : 0;
    S.device_bytes = int64_t(P.mem.total());
    S.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    P.built = true;
    return plan.release();
}

}  // namespace

extern "C" {

int32_t h3d_version(void) { return H3D_VERSION; }

const char *h3d_last_error(void) { return g_last_error.c_str(); }

void h3d_config_init(h3d_config *cfg) {
    if (!cfg)
        return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->kernel = H3D_LAPLACE;
    cfg->kernel_param = 1.0;
    cfg->leaf_size = 64;
    cfg->tol = 1e-8;
    cfg->factor_dtype = H3D_F64;
    cfg->max_rank = 0;
    cfg->max_depth = 10;
    cfg->box_side = 0.0;
    cfg->workspace_bytes = 0;
    cfg->flags = 0;
}

h3d_status h3d_build(const double *points, int64_t n, const h3d_config *cfg,
                     const h3d_allocator *alloc, void *hip_stream, h3d_plan **out) {
    if (!out)
        return invalid("out must not be NULL");
    *out = nullptr;
    h3d_status st = check_config(cfg, alloc);
    if (st != H3D_OK)
        return st;
    if (!points)
        return invalid("points must not be NULL");
    if (n < 1 || n > int64_t(0x7fffffff) - 1)
        return invalid("n must be in [1, 2^31 - 2]");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    h3d_plan *plan = nullptr;
    st = guarded([&] { plan = build_plan(points, n, *cfg, alloc, s, false); });
    if (st != H3D_OK) {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        delete plan;
        return st;
    }
    reg_add(plan, kOwnPlan);
    *out = plan;
    return H3D_OK;
}

h3d_status h3d_build_batch(int32_t nprob, const double *const *points, const int64_t *n,
                           const h3d_config *cfg, const h3d_allocator *alloc, void *hip_stream,
                           h3d_plan **out) {
    if (!out)
        return invalid("out must not be NULL");
    *out = nullptr;
    if (nprob < 1)
        return invalid("nprob must be >= 1");
    if (!points || !n)
        return invalid("points and n must not be NULL");
    h3d_status st = check_config(cfg, alloc);
    if (st != H3D_OK)
        return st;
    if (cfg->flags & H3D_FLAG_LU_FORM)
        return g_last_error = "the batch launches carry the explicit-factor kernels: "
                              "H3D_FLAG_LU_FORM is not available for batches",
               H3D_ENOTIMPL;
    for (int32_t i = 0; i < nprob; ++i) {
        if (!points[i])
            return invalid("points[" + std::to_string(i) + "] is NULL");
        if (n[i] < 1 || n[i] > int64_t(0x7fffffff) - 1)
            return invalid("n[" + std::to_string(i) + "] must be in [1, 2^31 - 2]");
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    h3d_plan *bp = nullptr;
    st = guarded([&] {
        const auto t0 = std::chrono::steady_clock::now();
        bp = new h3d_plan();
        bp->batch = new h3d::BatchState();
        h3d::Plan &P = bp->P;
        P.cfg = *cfg;
        H3D_HIP(hipGetDevice(&P.device));
        P.mem.configure(alloc, s);
        P.factor_dtype = cfg->factor_dtype;
        h3d_stats &S = P.stats;
        S.factor_dtype = cfg->factor_dtype;
        for (int32_t i = 0; i < nprob; ++i) {
            bp->batch->subs.push_back(nullptr);
            h3d_plan *q = build_plan(points[i], n[i], *cfg, alloc, s, true);
            bp->batch->subs.back() = q;
            const h3d_stats &Q = q->P.stats;
            S.n += Q.n;
            S.depth = std::max(S.depth, Q.depth);
            S.n_far += Q.n_far;
            S.n_near += Q.n_near;
            for (int l = 0; l < H3D_MAX_LEVELS; ++l) {
                S.far_per_level[l] += Q.far_per_level[l];
                S.factor_bytes_per_level[l] += Q.factor_bytes_per_level[l];
            }
            S.rank_sum += Q.rank_sum;
            S.rank_max = std::max(S.rank_max, Q.rank_max);
            S.n_rank_capped += Q.n_rank_capped;
            S.factor_entries += Q.factor_entries;
            S.factor_bytes += Q.factor_bytes;
            S.near_pair_evals += Q.near_pair_evals;
            S.aca_ms += Q.aca_ms;
        }
        h3d::batch_setup(*bp, s);
        H3D_HIP(hipStreamSynchronize(s));
        P.n = S.n;
        S.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        P.built = true;
    });
    if (st != H3D_OK) {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        delete bp;
        return st;
    }
    reg_add(bp, kOwnPlan);
    for (h3d_plan *q : bp->batch->subs)
        reg_add(q, kMemberPlan);
    *out = bp;
    return H3D_OK;
}

h3d_status h3d_matvec_batch(h3d_plan *batch, const void *const *x, void *const *y, int64_t nrhs,
                            int32_t io_dtype, void *hip_stream) {
    if (const h3d_status ps = plan_status(batch); ps != H3D_OK)
        return ps;
    if (!batch->batch)
        return invalid("not a batch plan (built by h3d_build_batch)");
    if (!x || !y)
        return invalid("x and y must be host arrays of device pointers");
    const auto &subs = batch->batch->subs;
    for (size_t i = 0; i < subs.size(); ++i) {
        const int64_t ni = subs[i]->P.n;
        const h3d_status st = matvec_check(subs[i], x[i], y[i], nrhs, ni, ni, io_dtype);
        if (st != H3D_OK) {
            g_last_error = "problem " + std::to_string(i) + ": " + g_last_error;
            return st;
        }
    }
    return guarded([&] {
        DeviceScope ds(batch->P.device);
        h3d::batch_run(*batch, x, y, nrhs, io_dtype, static_cast<hipStream_t>(hip_stream));
    });
}

h3d_status h3d_batch_plan(h3d_plan *batch, int32_t i, h3d_plan **out) {
    if (!out)
        return invalid("out must not be NULL");
    *out = nullptr;
    if (const h3d_status ps = plan_status(batch); ps != H3D_OK)
        return ps;
    if (!batch->batch)
        return invalid("not a batch plan (built by h3d_build_batch)");
    if (i < 0 || size_t(i) >= batch->batch->subs.size())
        return invalid("problem index out of range");
    *out = batch->batch->subs[size_t(i)];
    return H3D_OK;
}

h3d_status h3d_batch_check(h3d_plan *batch, void *hip_stream) {
    if (const h3d_status ps = plan_status(batch); ps != H3D_OK)
        return ps;
    if (!batch->batch)
        return invalid("not a batch plan (built by h3d_build_batch)");
    bool failed = false;
    const h3d_status st = guarded([&] {
        DeviceScope ds(batch->P.device);
        failed = h3d::batch_wait_failed(*batch, static_cast<hipStream_t>(hip_stream));
    });
    if (st != H3D_OK)
        return st;
    if (failed)
        return g_last_error = "a dependency wait of the batch product gave up", H3D_EDEVICE;
    return H3D_OK;
}

h3d_status h3d_matvec(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                      int64_t ldy, int32_t io_dtype, void *hip_stream) {
    return matvec_common(plan, x, y, nrhs, ldx, ldy, io_dtype, hip_stream, false);
}

h3d_status h3d_matvec_adjoint(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                              int64_t ldy, int32_t io_dtype, void *hip_stream) {
    return matvec_common(plan, x, y, nrhs, ldx, ldy, io_dtype, hip_stream, true);
}

h3d_status h3d_graph_create(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                            int64_t ldy, int32_t io_dtype, int32_t adjoint, void *hip_stream,
                            h3d_graph **out) {
    if (!out)
        return invalid("out must not be NULL");
    *out = nullptr;
    h3d_status st = matvec_check(plan, x, y, nrhs, ldx, ldy, io_dtype);
    if (st != H3D_OK)
        return st;
    h3d_graph *g = nullptr;
    hipStream_t cs = nullptr;
    st = guarded([&] {
        h3d::Plan &P = plan->P;
        DeviceScope ds(P.device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        // eager run: allocates scratch and tables outside the capture
        h3d::matvec_run(P, x, y, nrhs, ldx, ldy, io_dtype, adjoint != 0, s);
        H3D_HIP(hipStreamSynchronize(s));
        g = new h3d_graph();
        g->plan = plan;
        const bool prof = P.prof.on;
        P.prof.on = false;
        H3D_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        H3D_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            h3d::matvec_run(P, x, y, nrhs, ldx, ldy, io_dtype, adjoint != 0, cs);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cs, &dead);
            if (dead)
                (void)hipGraphDestroy(dead);
            P.prof.on = prof;
            throw;
        }
        H3D_HIP(hipStreamEndCapture(cs, &g->graph));
        P.prof.on = prof;
        H3D_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        P.live_graphs += 1;
    });
    if (cs)
        (void)hipStreamDestroy(cs);
    if (st != H3D_OK) {
        if (g) {
            if (g->exec)
                (void)hipGraphExecDestroy(g->exec);
            if (g->graph)
                (void)hipGraphDestroy(g->graph);
            delete g;
        }
        return st;
    }
    reg_add(g, kGraph);
    *out = g;
    return H3D_OK;
}

h3d_status h3d_graph_create_batch(h3d_plan *batch, const void *const *x, void *const *y,
                                  int64_t nrhs, int32_t io_dtype, void *hip_stream,
                                  h3d_graph **out) {
    if (!out)
        return invalid("out must not be NULL");
    *out = nullptr;
    if (const h3d_status ps = plan_status(batch); ps != H3D_OK)
        return ps;
    if (!batch->batch)
        return invalid("not a batch plan (built by h3d_build_batch)");
    if (!x || !y)
        return invalid("x and y must be host arrays of device pointers");
    const auto &subs = batch->batch->subs;
    for (size_t i = 0; i < subs.size(); ++i) {
        const int64_t ni = subs[i]->P.n;
        const h3d_status st = matvec_check(subs[i], x[i], y[i], nrhs, ni, ni, io_dtype);
        if (st != H3D_OK) {
            g_last_error = "problem " + std::to_string(i) + ": " + g_last_error;
            return st;
        }
    }
    // the graph keeps the pointers: copies of the caller's arrays
    std::vector<const void *> xs(x, x + subs.size());
    std::vector<void *> ys(y, y + subs.size());
    h3d_graph *g = nullptr;
    hipStream_t cs = nullptr;
    h3d_status st = guarded([&] {
        h3d::Plan &P = batch->P;
        DeviceScope ds(P.device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        // eager run: scratch, descriptors and tables outside the capture
        h3d::batch_run(*batch, xs.data(), ys.data(), nrhs, io_dtype, s);
        H3D_HIP(hipStreamSynchronize(s));
        g = new h3d_graph();
        g->plan = batch;
        g->batch = true;
        std::vector<bool> prof(subs.size() + 1);
        prof[0] = P.prof.on;
        P.prof.on = false;
        for (size_t i = 0; i < subs.size(); ++i) {
            prof[i + 1] = subs[i]->P.prof.on;
            subs[i]->P.prof.on = false;
        }
        auto restore = [&] {
            P.prof.on = prof[0];
            for (size_t i = 0; i < subs.size(); ++i)
                subs[i]->P.prof.on = prof[i + 1];
        };
        H3D_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        H3D_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            h3d::batch_run(*batch, xs.data(), ys.data(), nrhs, io_dtype, cs);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cs, &dead);
            if (dead)
                (void)hipGraphDestroy(dead);
            restore();
            throw;
        }
        H3D_HIP(hipStreamEndCapture(cs, &g->graph));
        restore();
        H3D_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        P.live_graphs += 1;
        for (h3d_plan *q : subs)
            q->P.live_graphs += 1;
    });
    if (cs)
        (void)hipStreamDestroy(cs);
    if (st != H3D_OK) {
        if (g) {
            if (g->exec)
                (void)hipGraphExecDestroy(g->exec);
            if (g->graph)
                (void)hipGraphDestroy(g->graph);
            delete g;
        }
        return st;
    }
    reg_add(g, kGraph);
    *out = g;
    return H3D_OK;
}

h3d_status h3d_graph_launch(h3d_graph *graph, void *hip_stream) {
    if (!graph || reg_kind(graph) != kGraph || !graph->exec)
        return invalid("not a live graph (NULL or destroyed)");
    return guarded([&] {
        DeviceScope ds(graph->plan->P.device);
        H3D_HIP(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(hip_stream)));
    });
}

h3d_status h3d_graph_destroy(h3d_graph *graph) {
    if (!graph)
        return H3D_OK;
    if (reg_kind(graph) != kGraph)
        return invalid("not a live graph (already destroyed?)");
    reg_del(graph);
    return guarded([&] {
        // the plan outlives its graphs: h3d_destroy refuses a plan with live graphs
        graph->plan->P.live_graphs -= 1;
        if (graph->batch)
            for (h3d_plan *q : graph->plan->batch->subs)
                q->P.live_graphs -= 1;
        DeviceScope ds(graph->plan->P.device);
        (void)hipDeviceSynchronize();
        if (graph->exec)
            (void)hipGraphExecDestroy(graph->exec);
        if (graph->graph)
            (void)hipGraphDestroy(graph->graph);
        delete graph;
    });
}

h3d_status h3d_autotune(h3d_plan *plan, int64_t nrhs, void *hip_stream) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    if (plan->batch)
        return batch_plan_error();
    if (plan->P.in_batch)
        return invalid("the launch shapes of a batch member are fixed by its batch");
    if (nrhs < 1)
        return invalid("nrhs must be >= 1");
    if (plan->P.live_graphs > 0)
        return invalid("autotuning rebuilds work tables that captured graphs of this plan use: "
                       "destroy them first");
    return guarded([&] {
        DeviceScope ds(plan->P.device);
        h3d::autotune(plan->P, nrhs, static_cast<hipStream_t>(hip_stream));
    });
}

h3d_status h3d_get_stats(const h3d_plan *plan, h3d_stats *out) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    if (!out)
        return invalid("out must not be NULL");
    *out = plan->P.stats;
    out->device_bytes = int64_t(plan->P.mem.total());
    if (plan->batch)
        for (const h3d_plan *q : plan->batch->subs)
            out->device_bytes += int64_t(q->P.mem.total());
    return H3D_OK;
}

h3d_status h3d_export(const h3d_plan *plan, int32_t what, void *host_buf, size_t *bytes) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    if (plan->batch)
        return batch_plan_error();
    if (!bytes)
        return invalid("bytes must not be NULL");
    h3d::Plan &P = const_cast<h3d::Plan &>(plan->P);
    const int64_t nf = P.nfar;
    size_t need = 0;
    switch (what) {
    case H3D_EXPORT_PERM:
        need = size_t(P.n) * 8;
        break;
    case H3D_EXPORT_LEAF_OFF:
        need = P.h_leaf_off.size() * 8;
        break;
    case H3D_EXPORT_FAR:
        need = size_t(nf) * 6 * 8;
        break;
    case H3D_EXPORT_NEAR:
        need = size_t(P.nnear) * 3 * 8;
        break;
    case H3D_EXPORT_FACTORS_U:
    case H3D_EXPORT_FACTORS_V: {
        if (P.lu_form)
            return invalid("a pivot + LU form plan stores no explicit factors: export "
                           "H3D_EXPORT_LU");
        const int64_t ev = P.entries_v;
        need = size_t(what == H3D_EXPORT_FACTORS_V ? ev : P.stats.factor_entries - ev) * 8;
        break;
    }
    case H3D_EXPORT_PIVOTS:
        if (!P.blk_piv)
            return invalid("pivots were not kept (build with H3D_FLAG_KEEP_PIVOTS)");
        need = size_t(P.ncols) * 2 * 8;
        break;
    case H3D_EXPORT_LU:
        if (!P.lu_form)
            return invalid("H3D_EXPORT_LU needs a plan built with H3D_FLAG_LU_FORM");
        need = size_t(P.lu_sq) * 8;
        break;
    default:
        return invalid("unknown export id");
    }
    if (!host_buf) {
        *bytes = need;
        return H3D_OK;
    }
    if (*bytes < need)
        return invalid("host buffer too small");
    int64_t *o = static_cast<int64_t *>(host_buf);
    return guarded([&] {
        DeviceScope ds(P.device);
        hipStream_t s = nullptr;
        H3D_HIP(hipDeviceSynchronize());
        switch (what) {
        case H3D_EXPORT_PERM: {
            std::vector<int32_t> v(static_cast<size_t>(P.n));
            h3d::to_host(v.data(), P.perm, P.n, s);
            for (int64_t i = 0; i < P.n; ++i)
                o[i] = v[size_t(i)];
            break;
        }
        case H3D_EXPORT_LEAF_OFF:
            for (size_t i = 0; i < P.h_leaf_off.size(); ++i)
                o[i] = P.h_leaf_off[i];
            break;
        case H3D_EXPORT_FAR: {
            std::vector<int32_t> v(static_cast<size_t>(nf));
            int l = 1;
            for (int64_t b = 0; b < nf; ++b) {
                while (b >= P.lvl_blk[l + 1])
                    ++l;
                o[b] = l;
            }
            const int32_t *cols[5] = {P.blk_t, P.blk_s, P.blk_m, P.blk_n, P.blk_rank};
            for (int c = 0; c < 5; ++c) {
                h3d::to_host(v.data(), cols[c], nf, s);
                for (int64_t b = 0; b < nf; ++b)
                    o[(c + 1) * nf + b] = v[size_t(b)];
            }
            break;
        }
        case H3D_EXPORT_NEAR: {
            const int64_t nn = P.nnear, nleaf = h3d::pow8(P.L);
            std::vector<int32_t> ptr(static_cast<size_t>(nleaf) + 1);
            std::vector<int32_t> sv(static_cast<size_t>(nn));
            std::vector<int8_t> rv(static_cast<size_t>(nn));
            h3d::to_host(ptr.data(), P.near_ptr, nleaf + 1, s);
            h3d::to_host(sv.data(), P.near_s, nn, s);
            h3d::to_host(rv.data(), P.near_rel, nn, s);
            for (int64_t t = 0; t < nleaf; ++t)
                for (int32_t e = ptr[size_t(t)]; e < ptr[size_t(t) + 1]; ++e) {
                    o[e] = t;
                    o[nn + e] = sv[size_t(e)];
                    o[2 * nn + e] = rv[size_t(e)];
                }
            break;
        }
        case H3D_EXPORT_FACTORS_U:
        case H3D_EXPORT_FACTORS_V:
            h3d::export_factors(P, what == H3D_EXPORT_FACTORS_U ? 0 : 1,
                                static_cast<double *>(host_buf));
            break;
        case H3D_EXPORT_PIVOTS: {
            std::vector<int32_t> rank(static_cast<size_t>(nf));
            std::vector<int64_t> off(size_t(nf) + 1);
            h3d::to_host(rank.data(), P.blk_rank, nf, s);
            h3d::to_host(off.data(), P.blk_pivoff, nf + 1, s);
            std::vector<int32_t> piv(static_cast<size_t>(off[size_t(nf)]));
            h3d::to_host(piv.data(), P.blk_piv, off[size_t(nf)], s);
            int64_t c = 0;
            for (int64_t b = 0; b < nf; ++b)
                for (int k = 0; k < rank[size_t(b)]; ++k, ++c) {
                    o[c] = piv[size_t(off[size_t(b)] + 2 * k)];
                    o[P.ncols + c] = piv[size_t(off[size_t(b)] + 2 * k + 1)];
                }
            break;
        }
        case H3D_EXPORT_LU:
            h3d::export_lu(P, static_cast<double *>(host_buf));
            break;
        }
        *bytes = need;
    });
}

h3d_status h3d_destroy(h3d_plan *plan) {
    if (!plan)
        return H3D_OK;
    const int kind = reg_kind(plan);
    if (kind == kMemberPlan)
        return invalid("a problem of a batch belongs to its batch: destroy the batch");
    if (kind != kOwnPlan)
        return invalid("not a live plan (already destroyed?)");
    int graphs = plan->P.live_graphs;
    if (plan->batch)
        for (const h3d_plan *q : plan->batch->subs)
            graphs += q->P.live_graphs;
    if (graphs > 0)
        return invalid("the plan has " + std::to_string(graphs) +
                       " live graph(s): destroy them first");
    reg_del(plan);
    if (plan->batch)
        for (const h3d_plan *q : plan->batch->subs)
            reg_del(q);
    return guarded([&] {
        {
            DeviceScope ds(plan->P.device);
            (void)hipDeviceSynchronize();
        }
        delete plan;
    });
}

h3d_status h3d_solve_gmres(h3d_plan *plan, double diag, double scale, const double *f, double *x,
                           double rtol, int32_t restart, int32_t max_iter, void *hip_stream,
                           h3d_solve_info *info) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    if (plan->batch)
        return batch_plan_error();
    h3d::Plan &P = plan->P;
    if (!f || !x)
        return invalid("f and x must be device pointers");
    const uintptr_t fa = uintptr_t(f), xa = uintptr_t(x), nb = size_t(P.n) * 8;
    if (fa < xa + nb && xa < fa + nb)
        return invalid("f and x overlap");
    if (!(rtol > 0.0 && rtol < 1.0))
        return invalid("rtol must lie in (0, 1)");
    if (restart < 1 || restart > h3d::kMaxRestart)
        return invalid("restart must lie in [1, 256]");
    if (max_iter < 1)
        return invalid("max_iter must be >= 1");
    if (!std::isfinite(diag) || !std::isfinite(scale))
        return invalid("diag and scale must be finite");
    return guarded([&] {
        DeviceScope ds(P.device);
        const h3d::SolveResult r = h3d::solve_gmres(P, diag, scale, f, x, rtol, restart, max_iter,
                                                    static_cast<hipStream_t>(hip_stream));
        if (info) {
            info->iterations = r.iterations;
            info->cycles = r.cycles;
            info->converged = r.converged;
            info->rel_residual = r.rel_residual;
            info->est_residual = r.est_residual;
        }
    });
}

h3d_status h3d_dense_matvec(const double *points, int64_t n, int32_t kernel,
                            double kernel_param, const double *x, double *y, void *hip_stream) {
    if (n < 1)
        return invalid("n must be >= 1");
    if (!points || !x || !y)
        return invalid("points, x and y must be device pointers");
    if (kernel < H3D_LAPLACE || kernel > H3D_COS_R)
        return invalid("unknown kernel");
    if (!std::isfinite(kernel_param))
        return invalid("kernel_param must be finite");
    const uintptr_t xa = uintptr_t(x), ya = uintptr_t(y), nb = size_t(n) * 8;
    if (xa < ya + nb && ya < xa + nb)
        return invalid("x and y overlap");
    return guarded([&] {
        h3d::dense_matvec(points, n, kernel, kernel_param, x, y,
                          static_cast<hipStream_t>(hip_stream));
    });
}

h3d_status h3d_profile_enable(h3d_plan *plan, int32_t enable) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    return guarded([&] {
        plan->P.prof.collect();
        plan->P.prof.on = enable != 0;
        plan->P.prof.levels = enable >= 2;
    });
}

h3d_status h3d_profile_reset(h3d_plan *plan) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    return guarded([&] { plan->P.prof.reset(); });
}

h3d_status h3d_profile_read(h3d_plan *plan, h3d_kernel_profile *out, int32_t capacity,
                            int32_t *count) {
    if (const h3d_status ps = plan_status(plan); ps != H3D_OK)
        return ps;
    if (!count || (capacity > 0 && !out))
        return invalid("count (and out when capacity > 0) must not be NULL");
    return guarded([&] {
        h3d::Profiler &pr = plan->P.prof;
        pr.collect();
        const int32_t nk = int32_t(pr.names.size());
        *count = nk;
        for (int32_t i = 0; i < nk && i < capacity; ++i) {
            std::memset(out[i].name, 0, sizeof(out[i].name));
            std::strncpy(out[i].name, pr.names[size_t(i)].c_str(), sizeof(out[i].name) - 1);
            out[i].launches = pr.launches[size_t(i)];
            out[i].total_ms = pr.total_ms[size_t(i)];
            const double nl = double(std::max<int64_t>(pr.launches[size_t(i)], 1));
            out[i].bytes_per_launch = pr.bytes[size_t(i)] / nl;
            out[i].flops_per_launch = pr.flops[size_t(i)] / nl;
        }
    });
}

}  // extern "C"

// ---- h3d_matvec_noalloc ----------------------------------------------------
// Its scratch (the sorted input, the sorted sums and the stage-1 z values of
// a vector product) lives in this array instead of plan memory.  Each GPU
// holds its own copy from the module's load on that GPU until the process
// ends.  Host code never uses the array's name as an address: the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_addr.
static __device__ __align__(256) unsigned char scratch[H3D_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_addr;  // per device; nullptr until looked up

// Device address of `scratch` on the current device (dev), looked up on the
// first call for that device.
unsigned char *scratch_address(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0)
        h3d::fail(H3D_EDEVICE, "no current device");
    if (size_t(dev) >= g_scratch_addr.size())
        g_scratch_addr.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch_addr[size_t(dev)]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            h3d::fail(H3D_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                       hipGetErrorString(e));
        g_scratch_addr[size_t(dev)] = static_cast<unsigned char *>(p);
    }
    return g_scratch_addr[size_t(dev)];
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

h3d_status h3d_matvec_noalloc(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                              int64_t ldy, int32_t io_dtype, void *hip_stream) {
    const h3d_status st = matvec_check(plan, x, y, nrhs, ldx, ldy, io_dtype);
    if (st != H3D_OK)
        return st;
    h3d::Plan &P = plan->P;
    if (nrhs >= h3d::kBatchedMinRhs)
        return invalid("h3d_matvec_noalloc takes nrhs < " + std::to_string(h3d::kBatchedMinRhs) +
                       " (the matrix-core path of more right-hand sides keeps plan scratch)");
    const size_t xb = round256(sizeof(double) * size_t(P.n) * size_t(nrhs));
    const size_t zb = round256(sizeof(double) * size_t(h3d::vector_z_entries(P, nrhs)));
    const size_t need = 2 * xb + zb;
    if (need > size_t(H3D_NOALLOC_SCRATCH_BYTES))
        return invalid("h3d_matvec_noalloc: this product needs " + std::to_string(need) +
                       " bytes of scratch, more than the " +
                       std::to_string(size_t(H3D_NOALLOC_SCRATCH_BYTES)) +
                       " it holds; use h3d_matvec");
    return guarded([&] {
        DeviceScope ds(P.device);
        unsigned char *base = scratch_address(P.device);
        double *xp = reinterpret_cast<double *>(base);
        double *yn = reinterpret_cast<double *>(base + xb);
        double *z = reinterpret_cast<double *>(base + 2 * xb);
        // profiling would create events: off for this call
        const bool prof = P.prof.on;
        P.prof.on = false;
        try {
            h3d::matvec_vector(P, x, y, nrhs, ldx, ldy, io_dtype, false, xp, yn, z,
                               static_cast<hipStream_t>(hip_stream));
        } catch (...) {
            P.prof.on = prof;
            throw;
        }
        P.prof.on = prof;
    });
}

}  // extern "C"
