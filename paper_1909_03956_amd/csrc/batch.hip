// Batched persistent prediction (plans), HIP-graph capture of a planned
// prediction, and the tile-shape autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace swv;

struct swv_plan_s {
    swv_ctx ctx = nullptr;
    int64_t n_inst = 0;
    std::vector<BatchInst> direct, tree;
    std::vector<swv_tree> trees;      // held (one reference each) while the plan lives
    BatchInst* d_direct = nullptr;
    BatchInst* d_tree = nullptr;
    WorkItem* d_items_direct = nullptr;
    WorkItem* d_items_tree = nullptr;     // FP64 tree instances
    WorkItem* d_items_tree32 = nullptr;   // F32C tree instances
    unsigned n_items_direct = 0, n_items_tree = 0, n_items_tree32 = 0;
    Comp* d_pack = nullptr;
    unsigned* d_counters = nullptr;  // [0] direct, [1] tree FP64, [2] tree F32C
    int vpl = 2, block = 256, grid_direct = 0, grid_tree = 0, grid_tree32 = 0, max_comp = 0;
    int jmax = 1, smax = 1;           // largest J and segment depth of the trees
    int tree_walker = 0, tree_depth = 1;
    bool pruned = false;              // some tree is thresholded (leaves above level J)
    int tile_rows = 0;
    int64_t total_terms = 0;
    int refs = 1;  // graphs captured from this plan hold a reference
};

struct swv_graph_s {
    swv_plan plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <class T>
int dev_upload(const std::vector<T>& h, T** out) {
    *out = nullptr;
    const size_t bytes = std::max<size_t>(h.size() * sizeof(T), 64);
    hipError_t e = hipMalloc((void**)out, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(SWV_ENOMEM, "plan: device allocation of %zu bytes failed", bytes);
    }
    if (!h.empty()) {
        e = hipMemcpy(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "plan upload");
    }
    return SWV_OK;
}

void plan_release(swv_plan p) {
    if (--p->refs > 0) return;
    swv_ctx ctx = p->ctx;
    {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (void* q : {(void*)p->d_direct, (void*)p->d_tree, (void*)p->d_items_direct,
                        (void*)p->d_items_tree,
                        (void*)p->d_items_tree32, (void*)p->d_pack, (void*)p->d_counters})
            if (q) (void)hipFree(q);
    }
    for (swv_tree t : p->trees) (void)swv_tree_destroy(t);   // drops the plan's reference
    delete p;
    ctx_release(ctx);
}

void free_plan_device(swv_plan p) {
    for (void* q : {(void*)p->d_direct, (void*)p->d_tree, (void*)p->d_items_direct,
                    (void*)p->d_items_tree,
                        (void*)p->d_items_tree32, (void*)p->d_pack, (void*)p->d_counters})
        if (q) (void)hipFree(q);
}

// Enqueues the planned prediction on stream s.
hipError_t enqueue_plan(swv_plan p, hipStream_t s) {
    hipError_t e = launch_batch_ingest(s, p->d_direct, (int)p->direct.size(), p->max_comp,
                                       p->d_pack, p->ctx->d_status);
    if (e != hipSuccess) return e;
    e = launch_reset_counters(s, p->d_counters, 3);
    if (e != hipSuccess) return e;
    e = launch_batch_direct(s, p->vpl, p->block, p->grid_direct, p->d_direct, p->d_pack,
                            p->d_items_direct, p->n_items_direct, p->d_counters,
                            p->ctx->d_status);
    if (e != hipSuccess) return e;
    e = launch_batch_tree(s, p->tree_walker, p->tree_depth, SWV_FP64, p->grid_tree, p->d_tree, p->d_items_tree, p->n_items_tree, p->d_counters + 1,
                          p->ctx->d_status, p->pruned);
    if (e != hipSuccess) return e;
    return launch_batch_tree(s, p->tree_walker, p->tree_depth, SWV_F32C, p->grid_tree32,
                             p->d_tree, p->d_items_tree32, p->n_items_tree32,
                             p->d_counters + 2, p->ctx->d_status, p->pruned);
}

int check_instance(const swv_instance& I, int k) {
    if (I.route != SWV_ROUTE_DIRECT && I.route != SWV_ROUTE_TREE)
        return fail(SWV_EINVAL, "instance %d: bad route %d", k, I.route);
    if (I.sign != 1 && I.sign != -1)
        return fail(SWV_EDOMAIN, "instance %d: sign must be +1 or -1", k);
    if (I.n_vis < 0) return fail(SWV_EINVAL, "instance %d: negative n_vis", k);
    if (I.n_vis > 0 && (!I.u || !I.v || !I.w || !I.vis_out))
        return fail(SWV_EINVAL, "instance %d: null visibility pointer", k);
    if (I.route == SWV_ROUTE_DIRECT) {
        if (I.prec != SWV_FP64 && I.prec != SWV_F32C)
            return fail(SWV_EINVAL, "instance %d: bad precision %d", k, I.prec);
        if (I.n_comp < 0 || I.n_comp > INT32_MAX)
            return fail(SWV_EINVAL, "instance %d: bad n_comp", k);
        if (I.n_comp > 0 && (!I.l || !I.m || !I.flux))
            return fail(SWV_EINVAL, "instance %d: null component pointer", k);
    } else {
        if (!I.tree) return fail(SWV_EINVAL, "instance %d: null tree", k);
        if (I.prec != SWV_FP64 && I.prec != SWV_F32C)
            return fail(SWV_EINVAL, "instance %d: bad precision %d", k, I.prec);
        if (tree_walker(I.tree, 1) < 0)
            return fail(SWV_ENOTSUP,
                        "instance %d: J = %d with %d nested branchings: above the compiled "
                        "maxima (J %d, or %d branchings)",
                        k, I.tree->J, I.tree->max_branching, kTreeMaxJ, kTreeMaxSeg - 1);
    }
    return SWV_OK;
}

}  // namespace

extern "C" {

int swv_batch_plan(swv_ctx ctx, int n, const swv_instance* inst, swv_plan* out) {
    if (!out) return fail(SWV_EINVAL, "swv_batch_plan: null out");
    *out = nullptr;
    if (!ctx) return fail(SWV_EINVAL, "swv_batch_plan: null context");
    if (n < 0 || (n > 0 && !inst)) return fail(SWV_EINVAL, "swv_batch_plan: bad instance list");
    for (int k = 0; k < n; ++k) {
        const int rc = check_instance(inst[k], k);
        if (rc) return rc;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_batch_plan: cannot select device");
    swv_plan p = nullptr;
    try {
        p = new swv_plan_s();
        p->ctx = ctx;
        p->n_inst = n;
        p->vpl = ctx->per_lane[kFamDirect64][1];
        p->block = ctx->block[kFamDirect64][1];
        int64_t off = 0, total_rows = 0;
        std::vector<int64_t> cost_per_row_direct, cost_per_row_tree;
        for (int k = 0; k < n; ++k) {
            const swv_instance& I = inst[k];
            BatchInst b{};
            b.u = I.u;
            b.v = I.v;
            b.w = I.w;
            b.out = I.vis_out;
            b.n_vis = I.n_vis;
            b.prec = I.prec;
            b.sgn = (double)I.sign;
            total_rows += I.n_vis;
            if (I.route == SWV_ROUTE_DIRECT) {
                b.l = I.l;
                b.m = I.m;
                b.flux = I.flux;
                b.comp_offset = off;
                b.n_comp = (int)I.n_comp;
                off += I.n_comp;
                p->max_comp = std::max(p->max_comp, (int)I.n_comp);
                p->direct.push_back(b);
                cost_per_row_direct.push_back(std::max<int64_t>(I.n_comp, 1));
                p->total_terms += I.n_vis * I.n_comp;
            } else {
                const TRec* rec = nullptr;
                int rc = upload_tree(ctx, I.tree, &rec);
                if (rc) {
                    delete p;
                    return rc;
                }
                b.rec = rec;
                b.n_roots = (int)I.tree->n_roots;
                b.J = I.tree->J;
                p->jmax = std::max(p->jmax, b.J);
                p->smax = std::max(p->smax, I.tree->max_branching + 1);
                p->pruned = p->pruned || I.tree->thresholded;
                p->tree.push_back(b);
                cost_per_row_tree.push_back((int64_t)I.tree->records.size() + 1);
                p->total_terms += I.n_vis * I.tree->n_comp;
            }
        }
        // one traversal for all trees of the plan: the tuned one where it fits
        const bool level_ok = p->jmax <= kBatchTreeMaxJ, branch_ok = p->smax <= kTreeMaxSeg;
        const bool want_branch = ctx->per_lane[kFamTree][1] == 2;
        if (!p->tree.empty() && !level_ok && !branch_ok) {
            delete p;
            return fail(SWV_ENOTSUP,
                        "swv_batch_plan: no compiled traversal fits every tree (largest J %d, "
                        "segment depth %d)",
                        p->jmax, p->smax);
        }
        p->tree_walker = (branch_ok && (want_branch || !level_ok)) ? 1 : 0;
        p->tree_depth = p->tree_walker ? p->smax : p->jmax;
        if (p->pruned) {
            // thresholded trees: the branch walker compiled for leaves above level J
            if (!branch_ok) {
                delete p;
                return fail(SWV_ENOTSUP, "swv_batch_plan: a thresholded tree's branching is "
                                         "above the compiled maximum");
            }
            p->tree_walker = 1;
            p->tree_depth = kTreeMaxSeg;
        }

        // persistent grids: as many blocks as stay resident
        p->grid_direct = ctx->n_cu * batch_direct_blocks_per_cu(p->vpl, p->block);
        p->grid_tree = ctx->n_cu * (p->pruned ? batch_tree_pruned_blocks_per_cu(SWV_FP64)
                                              : batch_tree_blocks_per_cu(p->tree_walker,
                                                                         p->tree_depth, SWV_FP64));
        p->grid_tree32 = ctx->n_cu * (p->pruned ? batch_tree_pruned_blocks_per_cu(SWV_F32C)
                                                : batch_tree_blocks_per_cu(p->tree_walker,
                                                                           p->tree_depth, SWV_F32C));
        const int64_t waves = (int64_t)p->grid_direct * (p->block / 64);
        // about 16 items per resident wave, in whole wave tiles, at most 64 of them
        const int64_t unit = 64LL * p->vpl;
        int64_t tile = total_rows / std::max<int64_t>(1, 16 * waves);
        tile = std::max<int64_t>(unit, std::min<int64_t>(64 * unit, (tile + unit - 1) / unit * unit));
        p->tile_rows = (int)tile;

        struct Item {
            WorkItem w;
            int64_t cost;
        };
        auto make_items = [&](const std::vector<BatchInst>& list,
                              const std::vector<int64_t>& cpr, int64_t tile_rows) {
            std::vector<Item> items;
            for (size_t k = 0; k < list.size(); ++k)
                for (int64_t r = 0; r < list[k].n_vis; r += tile_rows) {
                    const int nr = (int)std::min<int64_t>(tile_rows, list[k].n_vis - r);
                    items.push_back(Item{WorkItem{r, (int)k, nr}, (int64_t)nr * cpr[k]});
                }
            // longest processing time first
            std::stable_sort(items.begin(), items.end(),
                             [](const Item& a, const Item& b) { return a.cost > b.cost; });
            std::vector<WorkItem> w;
            w.reserve(items.size());
            for (const Item& it : items) w.push_back(it.w);
            return w;
        };
        const std::vector<WorkItem> wd = make_items(p->direct, cost_per_row_direct, tile);
        const int64_t tree_tile = std::max<int64_t>(64, tile / p->vpl / 64 * 64);
        // tree items by precision (one launch each), keeping the cost order
        std::vector<WorkItem> wt, wt32;
        for (const WorkItem& it : make_items(p->tree, cost_per_row_tree, tree_tile))
            (p->tree[(size_t)it.inst].prec == SWV_F32C ? wt32 : wt).push_back(it);
        if (wd.size() > 0xffffffffull || wt.size() > 0xffffffffull || wt32.size() > 0xffffffffull) {
            delete p;
            return fail(SWV_ENOTSUP, "swv_batch_plan: too many work items");
        }
        p->n_items_direct = (unsigned)wd.size();
        p->n_items_tree = (unsigned)wt.size();
        p->n_items_tree32 = (unsigned)wt32.size();

        int rc = dev_upload(p->direct, &p->d_direct);
        if (!rc) rc = dev_upload(p->tree, &p->d_tree);
        if (!rc) rc = dev_upload(wd, &p->d_items_direct);
        if (!rc) rc = dev_upload(wt, &p->d_items_tree);
        if (!rc) rc = dev_upload(wt32, &p->d_items_tree32);
        if (!rc) {
            std::vector<Comp> none;
            none.resize((size_t)std::max<int64_t>(off, 1));
            hipError_t e = hipMalloc((void**)&p->d_pack, none.size() * sizeof(Comp));
            if (e != hipSuccess) {
                (void)hipGetLastError();
                p->d_pack = nullptr;
                rc = fail(SWV_ENOMEM, "swv_batch_plan: component buffer");
            }
        }
        if (!rc) {
            hipError_t e = hipMalloc((void**)&p->d_counters, 3 * sizeof(unsigned));
            if (e != hipSuccess) {
                (void)hipGetLastError();
                p->d_counters = nullptr;
                rc = fail(SWV_ENOMEM, "swv_batch_plan: counters");
            }
        }
        if (rc) {
            free_plan_device(p);
            delete p;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        if (p) {
            free_plan_device(p);
            delete p;
        }
        return fail(SWV_ENOMEM, "swv_batch_plan: host allocation failed");
    }
    ++ctx->refs;  // the plan keeps its context alive
    // and every tree whose device records it reads
    for (int k = 0; k < n; ++k)
        if (inst[k].route == SWV_ROUTE_TREE) {
            ++inst[k].tree->refs;
            p->trees.push_back(inst[k].tree);
        }
    *out = p;
    clear_error();
    return SWV_OK;
}

int swv_plan_stats(swv_plan p, swv_plan_stats_t* out) {
    if (!p || !out) return fail(SWV_EINVAL, "swv_plan_stats: null argument");
    out->n_instances = p->n_inst;
    out->n_items = (int64_t)p->n_items_direct + p->n_items_tree + p->n_items_tree32;
    out->total_terms = p->total_terms;
    out->tile_rows = p->tile_rows;
    out->grid_blocks = p->grid_direct;
    out->block_threads = p->block;
    return SWV_OK;
}

int swv_batch_run(swv_plan p) {
    if (!p) return fail(SWV_EINVAL, "swv_batch_run: null plan");
    DeviceGuard g(p->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_batch_run: cannot select device");
    const hipError_t e = enqueue_plan(p, p->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "swv_batch_run");
    return SWV_OK;
}

int swv_graph_capture(swv_plan p, swv_graph* out) {
    if (!out) return fail(SWV_EINVAL, "swv_graph_capture: null out");
    *out = nullptr;
    if (!p) return fail(SWV_EINVAL, "swv_graph_capture: null plan");
    DeviceGuard g(p->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_graph_capture: cannot select device");
    // capture on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is launched on the caller's
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e2 = enqueue_plan(p, cs);
        e = hipStreamEndCapture(cs, &graph);
        if (e2 != hipSuccess) e = e2;
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e, "graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    auto* gr = new (std::nothrow) swv_graph_s();
    if (!gr) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(SWV_ENOMEM, "swv_graph_capture: host allocation failed");
    }
    gr->plan = p;
    gr->graph = graph;
    gr->exec = exec;
    ++p->refs;  // the graph keeps its plan alive
    *out = gr;
    return SWV_OK;
}

int swv_graph_launch(swv_graph gr) {
    if (!gr) return fail(SWV_EINVAL, "swv_graph_launch: null graph");
    DeviceGuard g(gr->plan->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_graph_launch: cannot select device");
    const hipError_t e = hipGraphLaunch(gr->exec, gr->plan->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SWV_OK;
}

int swv_graph_destroy(swv_graph gr) {
    if (!gr) return SWV_OK;
    swv_plan p = gr->plan;
    {
        DeviceGuard g(p->ctx->device);
        (void)hipStreamSynchronize(p->ctx->stream);
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
    }
    delete gr;
    plan_release(p);
    return SWV_OK;
}

int swv_plan_destroy(swv_plan p) {
    if (!p) return SWV_OK;
    plan_release(p);
    return SWV_OK;
}

}  // extern "C"

// ------------------------------------------------------------- autotuner --
namespace {

const char* kFamilyNames[kFamilies] = {"direct_fp64", "direct_f32c", "tree", "adjoint", "grad"};

// Counter-based uniform numbers (splitmix64 finaliser) for tuning inputs.
__global__ void k_fill(double* x, int64_t n, uint64_t seed, double lo, double hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    x[i] = lo + (hi - lo) * (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    double* alloc(int64_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ptrs.push_back(p);
        return (double*)p;
    }
};

}  // namespace

extern "C" {

int swv_autotune(swv_ctx ctx, const char* cache_path, int flags) {
    if (!ctx) return fail(SWV_EINVAL, "swv_autotune: null context");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_autotune: cannot select device");
    // timed repetitions after one warm-up launch; the minimum is kept
    const int reps = (flags & 1) ? 2 : 5;
    const int64_t rows_of[2] = {int64_t(1) << 18, int64_t(1) << 22};
    // problem sizes of a wide-field major cycle: a few thousand components,
    // an image of about a thousand pixels
    const int n_comp = 2048, n_pix = 1024;
    const int n_par = n_comp > n_pix ? n_comp : n_pix;
    const hipStream_t s = ctx->stream;
    Scratch sc;
    const int64_t nmax = rows_of[1];
    double *u = sc.alloc(nmax), *v = sc.alloc(nmax), *w = sc.alloc(nmax), *y = sc.alloc(2 * nmax);
    double *l = sc.alloc(n_par), *m = sc.alloc(n_par), *f = sc.alloc(n_par), *nm = sc.alloc(n_par);
    double *out = sc.alloc(2 * nmax), *part = nullptr;
    double *g1 = sc.alloc(n_comp), *g2 = sc.alloc(n_comp), *g3 = sc.alloc(n_comp);
    if (!u || !v || !w || !y || !l || !m || !f || !nm || !out || !g1 || !g2 || !g3)
        return fail(SWV_ENOMEM, "swv_autotune: scratch allocation failed");
    struct F { double* p; int64_t n; double lo, hi; } fills[] = {
        {u, nmax, -1e5, 1e5}, {v, nmax, -1e5, 1e5}, {w, nmax, -2e4, 2e4}, {y, 2 * nmax, -1, 1},
        {l, n_par, -0.03, 0.03}, {m, n_par, -0.03, 0.03}, {f, n_par, 0.01, 1.0},
        {nm, n_par, -1e-3, -1e-6}};
    uint64_t seed = 12345;
    for (const F& x : fills)
        k_fill<<<dim3((unsigned)((x.n + 255) / 256)), dim3(256), 0, s>>>(x.p, x.n, seed++, x.lo, x.hi);
    Comp* comp = nullptr;
    {
        int rc = ensure(ctx, ctx->comp, sizeof(Comp) * n_comp);
        if (rc) return rc;
        comp = (Comp*)ctx->comp.p;
        hipError_t e = launch_ingest(s, n_comp, l, m, f, comp, ctx->d_status);
        if (e != hipSuccess) return hip_fail(e, "autotune ingest");
    }
    // a level-9 tree of 1,024 components in a 3 degree field
    std::vector<double> hl(1024), hm(1024), hf(1024);
    uint64_t st = 777;
    auto rnd = [&st]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(st >> 11) * (1.0 / 9007199254740992.0);
    };
    for (int i = 0; i < 1024; ++i) {
        hl[i] = (rnd() - 0.5) * 0.05;
        hm[i] = (rnd() - 0.5) * 0.05;
        hf[i] = 0.01 + rnd();
    }
    swv_tree tree = nullptr;
    int rc = swv_tree_build(9, 3.0, 0.5, 1024, hl.data(), hm.data(), hf.data(), &tree);
    if (rc) return rc;
    const TRec* rec = nullptr;
    rc = upload_tree(ctx, tree, &rec);
    if (rc) {
        swv_tree_destroy(tree);
        return rc;
    }
    const TreeArgs ta = tree_args(tree, rec);

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        swv_tree_destroy(tree);
        return fail(SWV_EHIP, "swv_autotune: event creation failed");
    }
    std::string report;
    int result = SWV_OK;
    for (int fam = 0; fam < kFamilies && result == SWV_OK; ++fam) {
        for (int cls = 0; cls < 2 && result == SWV_OK; ++cls) {
            const int64_t rows = rows_of[cls];
            float best = 1e30f;
            int best_pl = ctx->per_lane[fam][cls], best_bl = ctx->block[fam][cls];
            for (int pl : kPerLaneOptions) {
                for (int bl : kBlockOptions) {
                    if (!tune_valid(fam, pl, bl)) continue;
                    float tmin = 1e30f;
                    for (int r = 0; r <= reps; ++r) {
                        hipEventRecord(e0, s);
                        hipError_t e = hipSuccess;
                        if (fam == kFamDirect64 || fam == kFamDirect32) {
                            e = launch_direct(s, fam == kFamDirect64 ? SWV_FP64 : SWV_F32C, pl, bl,
                                              rows, u, v, w, comp, n_comp, -1, out, ctx->d_status);
                        } else if (fam == kFamTree) {
                            e = launch_tree(s, pl == 2 ? 1 : 0, bl, SWV_FP64, ta, rows, u, v, w,
                                            -1, out,
                                            ctx->d_status);
                        } else if (fam == kFamAdjoint) {
                            const int64_t tiles = (n_pix + (int64_t)pl * bl - 1) / ((int64_t)pl * bl);
                            const int64_t chunk = choose_chunk(rows, tiles, ctx->n_cu, adjoint_blocks_per_cu(SWV_FP64, pl, bl));
                            const int64_t nch = (rows + chunk - 1) / chunk;
                            rc = ensure(ctx, ctx->partial, 16 * (size_t)n_pix * nch);
                            if (rc) { result = rc; break; }
                            part = (double*)ctx->partial.p;
                            e = launch_adjoint(s, SWV_FP64, pl, bl, chunk, rows, u, v, w, y, n_pix,
                                               l, m, nm, -1, part, out);
                        } else {
                            int gblock = 128;
                            int64_t tiles = 1;
                            grad_tiling(pl, n_comp, &gblock, &tiles);
                            const int64_t chunk =
                                choose_chunk(rows, tiles, ctx->n_cu, grad_blocks_per_cu(pl, gblock));
                            const int64_t nch = (rows + chunk - 1) / chunk;
                            rc = ensure(ctx, ctx->partial, 32 * (size_t)n_comp * nch);
                            if (rc) { result = rc; break; }
                            part = (double*)ctx->partial.p;
                            e = launch_grad(s, pl, chunk, rows, u, v, w, y, comp, n_comp, -1, 1.0,
                                            part, g1, g2, g3);
                        }
                        hipEventRecord(e1, s);
                        if (e != hipSuccess) { result = hip_fail(e, "autotune launch"); break; }
                        if (hipEventSynchronize(e1) != hipSuccess) {
                            result = fail(SWV_EHIP, "autotune: event wait failed");
                            break;
                        }
                        float ms = 0.f;
                        hipEventElapsedTime(&ms, e0, e1);
                        if (r > 0) tmin = std::min(tmin, ms);   // r = 0 warms up
                    }
                    if (result != SWV_OK) break;
                    char line[160];
                    snprintf(line, sizeof line,
                             "    {\"family\": %d, \"name\": \"%s\", \"size_class\": %d, "
                             "\"per_lane\": %d, \"block\": %d, \"ms\": %.5f},\n",
                             fam, kFamilyNames[fam], cls, pl, bl, tmin);
                    report += line;
                    if (tmin < best) {
                        best = tmin;
                        best_pl = pl;
                        best_bl = bl;
                    }
                }
                if (result != SWV_OK) break;
            }
            ctx->per_lane[fam][cls] = best_pl;
            ctx->block[fam][cls] = best_bl;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    swv_tree_destroy(tree);
    if (result != SWV_OK) return result;
    if (cache_path) {
        FILE* fh = fopen(cache_path, "w");
        if (!fh) return fail(SWV_EINVAL, "swv_autotune: cannot write %s", cache_path);
        hipDeviceProp_t prop;
        const char* arch = hipGetDeviceProperties(&prop, ctx->device) == hipSuccess
                               ? prop.gcnArchName : "unknown";
        fprintf(fh, "{\n  \"format\": \"swvis-tune-1\",\n  \"arch\": \"%s\",\n  \"n_cu\": %d,\n",
                arch, ctx->n_cu);
        fprintf(fh, "  \"chosen\": [\n");
        for (int fam = 0; fam < kFamilies; ++fam)
            for (int cls = 0; cls < 2; ++cls)
                fprintf(fh,
                        "    {\"family\": %d, \"name\": \"%s\", \"size_class\": %d, "
                        "\"per_lane\": %d, \"block\": %d}%s\n",
                        fam, kFamilyNames[fam], cls, ctx->per_lane[fam][cls],
                        ctx->block[fam][cls], (fam == kFamilies - 1 && cls == 1) ? "" : ",");
        fprintf(fh, "  ],\n  \"timings\": [\n");
        if (report.size() >= 2) report.erase(report.size() - 2);  // trailing ",\n"
        fprintf(fh, "%s\n  ]\n}\n", report.c_str());
        fclose(fh);
    }
    return SWV_OK;
}

int swv_tune_load(swv_ctx ctx, const char* cache_path) {
    if (!ctx || !cache_path) return fail(SWV_EINVAL, "swv_tune_load: null argument");
    FILE* fh = fopen(cache_path, "r");
    if (!fh) return fail(SWV_EINVAL, "swv_tune_load: cannot read %s", cache_path);
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, fh)) > 0) text.append(buf, n);
    fclose(fh);
    if (text.find("\"swvis-tune-1\"") == std::string::npos)
        return fail(SWV_EINVAL, "swv_tune_load: %s is not a tuning table", cache_path);
    const size_t a = text.find("\"chosen\"");
    const size_t b = text.find("\"timings\"");
    if (a == std::string::npos) return fail(SWV_EINVAL, "swv_tune_load: no table in %s", cache_path);
    const std::string chosen = text.substr(a, b == std::string::npos ? std::string::npos : b - a);
    int table_pl[kFamilies][2], table_bl[kFamilies][2];
    std::memcpy(table_pl, ctx->per_lane, sizeof table_pl);
    std::memcpy(table_bl, ctx->block, sizeof table_bl);
    size_t pos = 0;
    int count = 0;
    while ((pos = chosen.find("{\"family\":", pos)) != std::string::npos) {
        int fam = -1, cls = -1, pl = 0, bl = 0;
        const char* q = chosen.c_str() + pos;
        const char* pf = std::strstr(q, "\"family\":");
        const char* pc = std::strstr(q, "\"size_class\":");
        const char* pp = std::strstr(q, "\"per_lane\":");
        const char* pb = std::strstr(q, "\"block\":");
        if (!pf || !pc || !pp || !pb || sscanf(pf, "\"family\": %d", &fam) != 1 ||
            sscanf(pc, "\"size_class\": %d", &cls) != 1 ||
            sscanf(pp, "\"per_lane\": %d", &pl) != 1 || sscanf(pb, "\"block\": %d", &bl) != 1 ||
            cls < 0 || cls > 1 || !tune_valid(fam, pl, bl))
            return fail(SWV_EINVAL, "swv_tune_load: bad entry in %s", cache_path);
        table_pl[fam][cls] = pl;
        table_bl[fam][cls] = bl;
        ++count;
        ++pos;
    }
    if (count == 0) return fail(SWV_EINVAL, "swv_tune_load: empty table in %s", cache_path);
    std::memcpy(ctx->per_lane, table_pl, sizeof table_pl);
    std::memcpy(ctx->block, table_bl, sizeof table_bl);
    return SWV_OK;
}

}  // extern "C"
