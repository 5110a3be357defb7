// Major cycles as one HIP graph (section 2.2: predict, subtract, image; the
// chi^2 gradients beside them).  An instance is one channel x pointing with
// its observed visibilities; every cycle runs, in one capture:
//   1. the batched persistent prediction of every instance (direct sums and
//      wavelet trees, one launch per route, FP64);
//   2. per instance: the subtract step with chi^2, the residual image on the
//      instance's pixel set (the exact adjoint) and, for a direct instance,
//      the chi^2 gradients of its components.
// The model of an instance changes from cycle to cycle.  Everything that
// depends on it is read on the device: component counts and pointers, the
// tree's root count and level from the instance descriptors, the tree records
// from a buffer sized for the largest model the instance accepts, the order
// of the work items from their list.  Grids and tilings are fixed by those
// capacities.  A new model is therefore an upload before the next replay,
// never a new capture.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.h"

using namespace swv;

struct swv_cycle_s {
    swv_ctx ctx = nullptr;
    std::vector<swv_cycle_instance> spec;
    std::vector<int> slot;                  // index of instance k in `direct` or `tree`
    std::vector<int64_t> cost;              // per-row cost of instance k's current model
    std::vector<BatchInst> direct, tree;    // host copies of the device descriptors
    std::vector<int> direct_inst, tree_inst;   // instance of each descriptor
    std::vector<WorkItem> items_direct, items_tree;
    std::vector<int64_t> rec_cap;           // per tree descriptor: record capacity
    BatchInst* d_direct = nullptr;
    BatchInst* d_tree = nullptr;
    WorkItem* d_items_direct = nullptr;
    WorkItem* d_items_tree = nullptr;
    Comp* d_pack = nullptr;
    TRec* d_rec = nullptr;
    unsigned* d_counters = nullptr;
    void* d_partial = nullptr;
    double* d_chi2_part = nullptr;
    // pinned host mirrors of the descriptors and work items, for async uploads
    void* h_mirror = nullptr;
    size_t mirror_bytes = 0;
    hipEvent_t up_event = nullptr;
    bool up_pending = false;
    bool dirty = true;
    int vpl = 2, block = 64, grid_direct = 0, grid_tree = 0, walker = 0, depth = 1;
    int max_comp_cap = 0;
    int64_t tile_rows = 64, tree_tile = 64;   // rows per work item, fixed at creation
    std::vector<AdjointShape> adj;          // per instance
    std::vector<int> gcpl;                  // per instance: gradient components per lane
    std::vector<int64_t> gchunk;            // per instance: gradient row chunk
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <class T>
int dev_alloc(T** p, size_t count) {
    *p = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 64);
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SWV_ENOMEM, "swv_cycle_create: device allocation of %zu bytes failed", bytes);
    }
    return SWV_OK;
}

void free_cycle(swv_cycle cy) {
    if (cy->exec) (void)hipGraphExecDestroy(cy->exec);
    if (cy->graph) (void)hipGraphDestroy(cy->graph);
    for (void* q : {(void*)cy->d_direct, (void*)cy->d_tree, (void*)cy->d_items_direct,
                    (void*)cy->d_items_tree, (void*)cy->d_pack, (void*)cy->d_rec,
                    (void*)cy->d_counters, cy->d_partial, (void*)cy->d_chi2_part})
        if (q) (void)hipFree(q);
    if (cy->h_mirror) (void)hipHostFree(cy->h_mirror);
    if (cy->up_event) (void)hipEventDestroy(cy->up_event);
}

int check_spec(const swv_cycle_instance& I, int k) {
    if (I.route != SWV_ROUTE_DIRECT && I.route != SWV_ROUTE_TREE)
        return fail(SWV_EINVAL, "cycle instance %d: bad route %d", k, I.route);
    if (I.sign != 1 && I.sign != -1)
        return fail(SWV_EDOMAIN, "cycle instance %d: sign must be +1 or -1", k);
    if (I.n_vis < 0 || I.n_pix < 0 || I.comp_cap < 0 || I.comp_cap > INT32_MAX)
        return fail(SWV_EINVAL, "cycle instance %d: bad size", k);
    if (I.n_vis > 0 && (!I.u || !I.v || !I.w || !I.vis_obs || !I.vis_model || !I.resid))
        return fail(SWV_EINVAL, "cycle instance %d: null visibility pointer", k);
    if (!I.chi2) return fail(SWV_EINVAL, "cycle instance %d: null chi2", k);
    if (I.n_pix > 0 && (!I.pix_l || !I.pix_m || !I.pix_nm1 || !I.image))
        return fail(SWV_EINVAL, "cycle instance %d: null pixel pointer", k);
    if (!std::isfinite(I.inv_sigma2))
        return fail(SWV_EDOMAIN, "cycle instance %d: bad inv_sigma2", k);
    const int ng = (I.d_flux != nullptr) + (I.d_l != nullptr) + (I.d_m != nullptr);
    if (ng != 0 && ng != 3)
        return fail(SWV_EINVAL, "cycle instance %d: give all three gradient outputs or none", k);
    if (ng && I.route != SWV_ROUTE_DIRECT)
        return fail(SWV_EINVAL, "cycle instance %d: gradients are for direct instances", k);
    if (I.route == SWV_ROUTE_TREE && (I.tree_level_cap < 1 || I.tree_level_cap > SWV_MAX_LEVEL))
        return fail(SWV_EDOMAIN, "cycle instance %d: tree_level_cap outside 1 .. %d", k,
                    SWV_MAX_LEVEL);
    return SWV_OK;
}

// Work items of the instances of one route: row tiles, longest processing
// time first for the current models.
void order_items(swv_cycle cy, const std::vector<int>& insts, int64_t tile_rows,
                 std::vector<WorkItem>& items) {
    struct Item {
        WorkItem w;
        int64_t cost;
    };
    std::vector<Item> all;
    for (size_t d = 0; d < insts.size(); ++d) {
        const int k = insts[d];
        const int64_t n = cy->spec[k].n_vis;
        for (int64_t r = 0; r < n; r += tile_rows) {
            const int nr = (int)std::min<int64_t>(tile_rows, n - r);
            all.push_back(Item{WorkItem{r, (int)d, nr}, (int64_t)nr * cy->cost[k]});
        }
    }
    std::stable_sort(all.begin(), all.end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    items.clear();
    for (const Item& it : all) items.push_back(it.w);
}

// Uploads changed descriptors and the new work order on the context's stream.
int upload(swv_cycle cy) {
    if (!cy->dirty) return SWV_OK;
    hipError_t e = hipSuccess;
    if (cy->up_pending) {
        e = hipEventSynchronize(cy->up_event);   // the mirror is free again
        if (e != hipSuccess) return hip_fail(e, "swv_cycle: previous upload");
        cy->up_pending = false;
    }
    char* m = (char*)cy->h_mirror;
    const size_t bd = cy->direct.size() * sizeof(BatchInst), bt = cy->tree.size() * sizeof(BatchInst);
    const size_t bid = cy->items_direct.size() * sizeof(WorkItem),
                 bit = cy->items_tree.size() * sizeof(WorkItem);
    if (bd) std::memcpy(m, cy->direct.data(), bd);
    if (bt) std::memcpy(m + bd, cy->tree.data(), bt);
    if (bid) std::memcpy(m + bd + bt, cy->items_direct.data(), bid);
    if (bit) std::memcpy(m + bd + bt + bid, cy->items_tree.data(), bit);
    const hipStream_t s = cy->ctx->stream;
    if (bd) e = hipMemcpyAsync(cy->d_direct, m, bd, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && bt) e = hipMemcpyAsync(cy->d_tree, m + bd, bt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && bid)
        e = hipMemcpyAsync(cy->d_items_direct, m + bd + bt, bid, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && bit)
        e = hipMemcpyAsync(cy->d_items_tree, m + bd + bt + bid, bit, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(cy->up_event, s);
    if (e != hipSuccess) return hip_fail(e, "swv_cycle: descriptor upload");
    cy->up_pending = true;
    cy->dirty = false;
    return SWV_OK;
}

hipError_t enqueue_cycle(swv_cycle cy, hipStream_t s) {
    swv_ctx ctx = cy->ctx;
    hipError_t e = launch_batch_ingest(s, cy->d_direct, (int)cy->direct.size(), cy->max_comp_cap,
                                       cy->d_pack, ctx->d_status);
    if (e != hipSuccess) return e;
    e = launch_reset_counters(s, cy->d_counters, 2);
    if (e != hipSuccess) return e;
    e = launch_batch_direct(s, cy->vpl, cy->block, cy->grid_direct, cy->d_direct, cy->d_pack,
                            cy->d_items_direct, (unsigned)cy->items_direct.size(),
                            cy->d_counters, ctx->d_status);
    if (e != hipSuccess) return e;
    e = launch_batch_tree(s, cy->walker, cy->depth, SWV_FP64, cy->grid_tree, cy->d_tree, cy->d_items_tree, (unsigned)cy->items_tree.size(),
                          cy->d_counters + 1, ctx->d_status);
    if (e != hipSuccess) return e;
    for (size_t k = 0; k < cy->spec.size(); ++k) {
        const swv_cycle_instance& I = cy->spec[k];
        e = launch_residual(s, I.n_vis, I.vis_obs, I.vis_model, I.inv_sigma2, I.resid,
                            cy->d_chi2_part, I.chi2);
        if (e != hipSuccess) return e;
        if (I.n_pix > 0) {
            const AdjointShape& a = cy->adj[k];
            e = launch_adjoint(s, SWV_FP64, a.ppl, a.block, a.chunk, I.n_vis, I.u, I.v, I.w,
                               I.resid, I.n_pix, I.pix_l, I.pix_m, I.pix_nm1, I.sign,
                               cy->d_partial, I.image);
            if (e != hipSuccess) return e;
        }
        if (I.d_flux && I.comp_cap > 0) {
            const int d = cy->slot[k];
            e = launch_grad(s, cy->gcpl[k], cy->gchunk[k], I.n_vis, I.u, I.v, I.w, I.resid,
                            cy->d_pack + cy->direct[d].comp_offset, I.comp_cap, I.sign,
                            -2.0 * I.inv_sigma2, (double*)cy->d_partial, I.d_flux, I.d_l, I.d_m,
                            &cy->d_direct[d].n_comp);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int swv_cycle_create(swv_ctx ctx, int n, const swv_cycle_instance* inst, swv_cycle* out) {
    if (!out) return fail(SWV_EINVAL, "swv_cycle_create: null out");
    *out = nullptr;
    if (!ctx) return fail(SWV_EINVAL, "swv_cycle_create: null context");
    if (n < 0 || (n > 0 && !inst)) return fail(SWV_EINVAL, "swv_cycle_create: bad instance list");
    for (int k = 0; k < n; ++k) {
        const int rc = check_spec(inst[k], k);
        if (rc) return rc;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_cycle_create: cannot select device");
    swv_cycle cy = nullptr;
    try {
        cy = new swv_cycle_s();
        cy->ctx = ctx;
        cy->spec.assign(inst, inst + n);
        cy->slot.assign(n, -1);
        cy->cost.assign(n, 1);
        cy->adj.resize(n);
        cy->gcpl.assign(n, 1);
        cy->gchunk.assign(n, 1);
        cy->vpl = ctx->per_lane[kFamDirect64][1];
        cy->block = ctx->block[kFamDirect64][1];
        int64_t comp_off = 0, rec_off = 0, rows = 0;
        int jcap = 1;
        for (int k = 0; k < n; ++k) {
            const swv_cycle_instance& I = inst[k];
            BatchInst b{};
            b.u = I.u;
            b.v = I.v;
            b.w = I.w;
            b.out = I.vis_model;
            b.n_vis = I.n_vis;
            b.prec = SWV_FP64;
            b.sgn = (double)I.sign;
            rows += I.n_vis;
            if (I.route == SWV_ROUTE_DIRECT) {
                b.comp_offset = comp_off;
                b.n_comp = 0;              // no model until swv_cycle_set_components
                comp_off += I.comp_cap;
                cy->max_comp_cap = std::max(cy->max_comp_cap, (int)I.comp_cap);
                cy->slot[k] = (int)cy->direct.size();
                cy->direct.push_back(b);
                cy->direct_inst.push_back(k);
            } else {
                // a level-j node exists only above a leaf: at most J records per leaf, plus
                // the roots
                const int64_t cap = std::max<int64_t>(1, I.comp_cap) * I.tree_level_cap + 12;
                if ((uint64_t)cap * sizeof(TRec) > kMaxRecordBytes) {
                    delete cy;
                    return fail(SWV_ENOTSUP, "swv_cycle_create: instance %d: %lld records exceed the "
                                "traversal's %zu-byte stream limit", k, (long long)cap,
                                (size_t)kMaxRecordBytes);
                }
                b.rec = nullptr;           // set below, once the record buffer exists
                b.comp_offset = rec_off;   // offset into the record buffer
                b.n_roots = 0;             // no model until swv_cycle_set_tree
                b.J = 1;
                rec_off += cap;
                jcap = std::max(jcap, I.tree_level_cap);
                cy->rec_cap.push_back(cap);
                cy->slot[k] = (int)cy->tree.size();
                cy->tree.push_back(b);
                cy->tree_inst.push_back(k);
            }
        }
        // one traversal for every tree of the cycle: the level walker up to its
        // largest J, else the branch walker at its deepest segment count
        cy->walker = jcap <= kBatchTreeMaxJ ? 0 : 1;
        cy->depth = cy->walker == 0 ? jcap : kTreeMaxSeg;
        cy->grid_direct = ctx->n_cu * batch_direct_blocks_per_cu(cy->vpl, cy->block);
        cy->grid_tree = ctx->n_cu * batch_tree_blocks_per_cu(cy->walker, cy->depth, SWV_FP64);
        const int64_t waves = (int64_t)cy->grid_direct * (cy->block / 64);
        const int64_t unit = 64LL * cy->vpl;
        int64_t tile = rows / std::max<int64_t>(1, 16 * waves);
        tile = std::max<int64_t>(unit, std::min<int64_t>(64 * unit, (tile + unit - 1) / unit * unit));
        cy->tile_rows = tile;
        cy->tree_tile = std::max<int64_t>(64, tile / cy->vpl / 64 * 64);
        order_items(cy, cy->direct_inst, cy->tile_rows, cy->items_direct);
        order_items(cy, cy->tree_inst, cy->tree_tile, cy->items_tree);
        if (cy->items_direct.size() > 0xffffffffull || cy->items_tree.size() > 0xffffffffull) {
            delete cy;
            return fail(SWV_ENOTSUP, "swv_cycle_create: too many work items");
        }
        // shapes of the per-instance image and gradient steps, and their scratch
        size_t partial = 64;
        int64_t res_blocks = 1;
        for (int k = 0; k < n; ++k) {
            const swv_cycle_instance& I = inst[k];
            res_blocks = std::max<int64_t>(res_blocks, residual_blocks(I.n_vis));
            if (I.n_pix > 0) {
                cy->adj[k] = adjoint_shape(ctx, I.n_vis, I.n_pix, SWV_FP64);
                partial = std::max(partial, adjoint_partial_bytes(cy->adj[k], I.n_pix));
            }
            if (I.d_flux && I.comp_cap > 0) {
                const int cpl = ctx->per_lane[kFamGrad][size_class(I.n_vis)];
                int gblock = 128;
                int64_t tiles = 1;
                grad_tiling(cpl, I.comp_cap, &gblock, &tiles);
                const int64_t chunk =
                    choose_chunk(I.n_vis, tiles, ctx->n_cu, grad_blocks_per_cu(cpl, gblock));
                const int64_t nch = I.n_vis > 0 ? (I.n_vis + chunk - 1) / chunk : 1;
                cy->gcpl[k] = cpl;
                cy->gchunk[k] = chunk;
                partial = std::max(partial, 32 * (size_t)I.comp_cap * (size_t)nch);
            }
        }
        int rc = dev_alloc(&cy->d_direct, cy->direct.size());
        if (!rc) rc = dev_alloc(&cy->d_tree, cy->tree.size());
        if (!rc) rc = dev_alloc(&cy->d_items_direct, cy->items_direct.size());
        if (!rc) rc = dev_alloc(&cy->d_items_tree, cy->items_tree.size());
        if (!rc) rc = dev_alloc(&cy->d_pack, (size_t)std::max<int64_t>(comp_off, 1));
        if (!rc) rc = dev_alloc(&cy->d_rec, (size_t)std::max<int64_t>(rec_off, 1));
        if (!rc) rc = dev_alloc(&cy->d_counters, 2);
        if (!rc) rc = dev_alloc((char**)&cy->d_partial, partial);
        if (!rc) rc = dev_alloc(&cy->d_chi2_part, (size_t)res_blocks);
        if (!rc) {
            cy->mirror_bytes = (cy->direct.size() + cy->tree.size()) * sizeof(BatchInst) +
                               (cy->items_direct.size() + cy->items_tree.size()) * sizeof(WorkItem) +
                               64;
            if (hipHostMalloc(&cy->h_mirror, cy->mirror_bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                cy->h_mirror = nullptr;
                rc = fail(SWV_ENOMEM, "swv_cycle_create: pinned host mirror");
            }
        }
        if (!rc && hipEventCreateWithFlags(&cy->up_event, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            cy->up_event = nullptr;
            rc = fail(SWV_EHIP, "swv_cycle_create: event");
        }
        if (rc) {
            free_cycle(cy);
            delete cy;
            return rc;
        }
        for (size_t d = 0; d < cy->tree.size(); ++d) cy->tree[d].rec = cy->d_rec + cy->tree[d].comp_offset;
    } catch (const std::bad_alloc&) {
        if (cy) {
            free_cycle(cy);
            delete cy;
        }
        return fail(SWV_ENOMEM, "swv_cycle_create: host allocation failed");
    }
    ++ctx->refs;   // the cycle keeps its context alive
    *out = cy;
    clear_error();
    return SWV_OK;
}

int swv_cycle_set_components(swv_cycle cy, int k, int64_t n_comp, const double* l,
                             const double* m, const double* flux) {
    if (!cy) return fail(SWV_EINVAL, "swv_cycle_set_components: null cycle");
    if (k < 0 || k >= (int)cy->spec.size() || cy->spec[k].route != SWV_ROUTE_DIRECT)
        return fail(SWV_EINVAL, "swv_cycle_set_components: %d is not a direct instance", k);
    if (n_comp < 0 || n_comp > cy->spec[k].comp_cap)
        return fail(SWV_EINVAL, "swv_cycle_set_components: %lld components, capacity %lld",
                    (long long)n_comp, (long long)cy->spec[k].comp_cap);
    if (n_comp > 0 && (!l || !m || !flux))
        return fail(SWV_EINVAL, "swv_cycle_set_components: null component pointer");
    BatchInst& b = cy->direct[(size_t)cy->slot[k]];
    b.l = l;
    b.m = m;
    b.flux = flux;
    b.n_comp = (int)n_comp;
    cy->cost[k] = std::max<int64_t>(n_comp, 1);
    order_items(cy, cy->direct_inst, cy->tile_rows, cy->items_direct);
    cy->dirty = true;
    return SWV_OK;
}

int swv_cycle_set_tree(swv_cycle cy, int k, swv_tree t) {
    if (!cy) return fail(SWV_EINVAL, "swv_cycle_set_tree: null cycle");
    if (k < 0 || k >= (int)cy->spec.size() || cy->spec[k].route != SWV_ROUTE_TREE)
        return fail(SWV_EINVAL, "swv_cycle_set_tree: %d is not a tree instance", k);
    if (!t) return fail(SWV_EINVAL, "swv_cycle_set_tree: null tree");
    if (t->thresholded)
        return fail(SWV_ENOTSUP, "swv_cycle_set_tree: thresholded trees are not supported in a "
                                 "captured cycle (its traversal is fixed at capture)");
    const int d = cy->slot[k];
    if (t->J > cy->spec[k].tree_level_cap)
        return fail(SWV_EINVAL, "swv_cycle_set_tree: J = %d above the instance's cap %d", t->J,
                    cy->spec[k].tree_level_cap);
    if ((int64_t)t->records.size() > cy->rec_cap[(size_t)d])
        return fail(SWV_EINVAL, "swv_cycle_set_tree: %zu records above the capacity %lld",
                    t->records.size(), (long long)cy->rec_cap[(size_t)d]);
    if (cy->walker == 1 && t->max_branching + 1 > cy->depth)
        return fail(SWV_ENOTSUP, "swv_cycle_set_tree: %d nested branchings, above %d",
                    t->max_branching, cy->depth - 1);
    DeviceGuard g(cy->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_cycle_set_tree: cannot select device");
    BatchInst& b = cy->tree[(size_t)d];
    if (!t->records.empty()) {
        // ordered after the work already on the stream, which may still read
        // the previous model's records; the wait keeps the copy's source valid
        hipError_t e = hipMemcpyAsync((void*)b.rec, t->records.data(),
                                      t->records.size() * sizeof(TRec), hipMemcpyHostToDevice,
                                      cy->ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(cy->ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "swv_cycle_set_tree: record upload");
    }
    b.n_roots = (int)t->n_roots;
    b.J = t->J;
    cy->cost[k] = (int64_t)t->records.size() + 1;
    order_items(cy, cy->tree_inst, cy->tree_tile, cy->items_tree);
    cy->dirty = true;
    return SWV_OK;
}

int swv_cycle_run(swv_cycle cy) {
    if (!cy) return fail(SWV_EINVAL, "swv_cycle_run: null cycle");
    DeviceGuard g(cy->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_cycle_run: cannot select device");
    int rc = upload(cy);
    if (rc) return rc;
    const hipError_t e = enqueue_cycle(cy, cy->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "swv_cycle_run");
    return SWV_OK;
}

int swv_cycle_capture(swv_cycle cy) {
    if (!cy) return fail(SWV_EINVAL, "swv_cycle_capture: null cycle");
    DeviceGuard g(cy->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_cycle_capture: cannot select device");
    hipError_t e = hipStreamSynchronize(cy->ctx->stream);   // a previous graph may be running
    if (e != hipSuccess) return hip_fail(e, "swv_cycle_capture");
    if (cy->exec) (void)hipGraphExecDestroy(cy->exec);
    if (cy->graph) (void)hipGraphDestroy(cy->graph);
    cy->exec = nullptr;
    cy->graph = nullptr;
    // capture on a private stream (the context's may be the legacy default
    // stream, which cannot be captured); replays go to the context's stream
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e2 = enqueue_cycle(cy, cs);
        e = hipStreamEndCapture(cs, &graph);
        if (e2 != hipSuccess) e = e2;
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e, "swv_cycle_capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    cy->graph = graph;
    cy->exec = exec;
    return SWV_OK;
}

int swv_cycle_launch(swv_cycle cy) {
    if (!cy) return fail(SWV_EINVAL, "swv_cycle_launch: null cycle");
    if (!cy->exec) return fail(SWV_EINVAL, "swv_cycle_launch: no captured graph");
    DeviceGuard g(cy->ctx->device);
    if (!g.ok) return fail(SWV_EHIP, "swv_cycle_launch: cannot select device");
    int rc = upload(cy);
    if (rc) return rc;
    const hipError_t e = hipGraphLaunch(cy->exec, cy->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SWV_OK;
}

int swv_cycle_destroy(swv_cycle cy) {
    if (!cy) return SWV_OK;
    swv_ctx ctx = cy->ctx;
    {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        free_cycle(cy);
    }
    delete cy;
    ctx_release(ctx);
    return SWV_OK;
}

}  // extern "C"
