// Host runtime behind the C ABI (pne.h): contexts, networks, batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "geometry.h"
#include "rankr.h"
#include "runtime.h"
#include "kernels.h"
#include "pne.h"

using namespace pne;

struct SiteLayout {
    std::vector<std::pair<std::vector<int>, std::vector<int>>> groups;  // leg dims -> sites, in dims order
    std::vector<int> colour;     // two-colouring of the site graph (meaningful when bipartite)
    bool bipartite = false;
    std::vector<int> slot_site;  // site of each global slot
};

struct PlanEntry {
    std::shared_ptr<Geometry> geo;
    std::map<int, std::shared_ptr<GeoPlan>> plans;  // by K, with bit 8 set for the complete-expansion mode
    std::shared_ptr<const SiteLayout> layout;       // built on first use
};

// Device instance tables of one plan, built and uploaded once per context:
// for every class instance and contraction step the absorbed slice's element
// offset from the network's slice base (excited legs at index 1) and its leg
// strides, and every instance's weight offset.  A batch only adds per-network
// slice and weight bases.
struct PlanTables {
    void *dev = nullptr;  // one allocation: records, then weight offsets
    size_t bytes = 0;
    struct Cls {
        const InstStep *tab;
        const int32_t *iw;
        int32_t n_inst, scalar, loop_e;
        int32_t wide_stride;  // a slice stride >= 2^24 (the entry-table path multiplies in 24 bits)
    };
    std::vector<Cls> cls;  // per class of the plan
};

struct pne_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    size_t used = 0;
    std::string err;
    std::mutex err_mu;  // a server's two threads may both report errors on the context
    std::multimap<uint64_t, PlanEntry> cache;
    std::mutex mu;
    double wall_khz = 100000.0;  // device wall clock rate (ticks per ms)
    double rank_ms[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // phases of the last profiled rank expansion
    void *staging = nullptr;     // pinned upload staging, reused by every batch creation
    size_t staging_bytes = 0;
    // Table uploads run on their own stream, so they never wait behind
    // kernels already queued on a batch's stream; the batch stream waits on
    // up_done instead, and the staging buffer is rewritten only once the
    // previous upload has completed.
    hipStream_t up_stream = nullptr;
    hipStream_t side_stream = nullptr;  // a batch's short BP launches, beside its wide-tile launch
    hipEvent_t up_done = nullptr;
    bool up_pending = false;
    // batch signature -> the variant pne_autotune chose (PNE_FLAG_AUTOTUNE)
    struct Tuned {
        uint32_t flags = 0;            // PNE_FLAG_GRAPH / PNE_FLAG_SEPARATE_REGAUGE
        int32_t small_sites = 0, tiles_in_flight = 0, reg_budget = 0;
        double ms = 0.0, default_ms = 0.0;  // best and default-variant run times when tuned
    };
    std::map<uint64_t, Tuned> tuned;
    std::unordered_map<const GeoPlan *, PlanTables> plan_tables;  // plans live as long as the context
};

struct pne_network {
    pne_ctx *ctx = nullptr;
    std::shared_ptr<Geometry> geo;
    std::vector<const double *> dptr;  // per site, device
    double *owned = nullptr;
    size_t owned_bytes = 0;
};

struct pne_batch {
    pne_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;  // stream every launch and copy of the batch is enqueued on
    std::vector<pne_network *> nets;
    pne_options opt{};
    std::vector<std::shared_ptr<GeoPlan>> plans;  // per net
    std::vector<int> site_base;                   // per net
    std::vector<int64_t> w_base;                  // per net
    std::vector<void *> allocs;
    // Fixed device region (the allocation-free entry point): tables and
    // buffers are placed there, results go to pageable host memory and
    // completion is a stream synchronisation (no events, one launch at a time).
    bool fixed = false;
    std::vector<char> h_host;
    size_t bytes = 0;
    DeviceBatch db;
    // Two pinned result slots: a batch may have two launches outstanding;
    // launch k copies its per-network state and results into slot k % 2 and
    // records done[k % 2]; waits take the launches in order.
    NetState *h_state_pinned = nullptr;     // slot of the current launch / wait
    NetResult *h_results_pinned = nullptr;
    NetState *h_state_slot[2] = {nullptr, nullptr};
    NetResult *h_results_slot[2] = {nullptr, nullptr};
    double *h_open_slot[2] = {nullptr, nullptr};  // open outputs of each slot's launch
    std::vector<int32_t> open_off;                 // per network: offset in the open outputs, -1 if closed
    int64_t open_total = 0;
    void *h_pinned = nullptr;               // the one pinned block holding both slots
    hipEvent_t done_slot[2] = {nullptr, nullptr};
    int64_t n_launched = 0, n_waited = 0;
    hipGraph_t graph = nullptr;             // captured launch sequence (PNE_FLAG_GRAPH)
    hipGraphExec_t graph_exec = nullptr;
    int first_chunk = 4;                 // sweeps before the first convergence check
    bool launched = false;
    bool waited = false;
    // per-kernel HIP-event timing (PNE_FLAG_PROFILE)
    struct TimedLaunch {
        int64_t launch;  // index of the batch launch the kernel belongs to
        int kid;
        hipEvent_t e0, e1;
    };
    std::vector<TimedLaunch> ev_used;
    std::vector<hipEvent_t> ev_pool;
    double kt_ms[KID_COUNT] = {0};
    int64_t kt_n[KID_COUNT] = {0};
    std::vector<NetState> h_state;  // state of the last waited launch, copied from its slot when needed
    int state_slot = -1;            // slot of the last waited launch while h_state lags it
    std::vector<FusedNet> h_fused;  // host copy of the persistent-block table
    std::vector<int32_t> paths;     // per network: PNE_PATH_* bits
    int64_t msg_total = 0;
    std::vector<int> msg_off;  // per global site
    std::vector<int> moff;     // per global slot, relative
};

namespace {

thread_local std::string g_tls_err;

pne_status fail(pne_ctx *ctx, pne_status st, const std::string &msg) {
    if (ctx) {
        std::lock_guard<std::mutex> lk(ctx->err_mu);
        ctx->err = msg;
    }
    g_tls_err = msg;
    return st;
}

pne_status hip_fail(pne_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, PNE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// Site layout of a geometry for the BP tables, built once per cached
// geometry: sites grouped by their leg-dimension tuple (tuple order), the
// two-colouring of the site graph, and each slot's site.
SiteLayout build_site_layout(const Geometry &g) {
    SiteLayout L;
    std::map<std::vector<int>, std::vector<int>> groups;
    for (int s = 0; s < g.n_sites; ++s)
        groups[std::vector<int>(g.dim.begin() + g.slot_base[s], g.dim.begin() + g.slot_base[s + 1])].push_back(s);
    L.groups.assign(groups.begin(), groups.end());
    L.slot_site.resize(g.slot_base[g.n_sites]);
    for (int s = 0; s < g.n_sites; ++s)
        for (int k = g.slot_base[s]; k < g.slot_base[s + 1]; ++k) L.slot_site[k] = s;
    L.colour.assign(g.n_sites, -1);
    bool bip = g.n_sites > 1;
    std::vector<std::vector<int>> adj(g.n_sites);
    for (int bb = 0; bb < g.n_bonds; ++bb) {
        adj[g.bu[bb]].push_back(g.bv[bb]);
        adj[g.bv[bb]].push_back(g.bu[bb]);
    }
    std::vector<int> queue;
    for (int s0 = 0; s0 < g.n_sites && bip; ++s0) {
        if (L.colour[s0] >= 0) continue;
        L.colour[s0] = 0;
        queue.assign(1, s0);
        for (size_t h = 0; h < queue.size() && bip; ++h) {
            const int u = queue[h];
            for (int v : adj[u]) {
                if (L.colour[v] < 0) {
                    L.colour[v] = 1 - L.colour[u];
                    queue.push_back(v);
                } else if (L.colour[v] == L.colour[u]) {
                    bip = false;
                    break;
                }
            }
        }
    }
    L.bipartite = bip;
    return L;
}

std::shared_ptr<GeoPlan> get_plan(pne_ctx *ctx, const std::shared_ptr<Geometry> &g, int K, bool full,
                                  std::string *err, std::shared_ptr<Geometry> *canon,
                                  std::shared_ptr<const SiteLayout> *layout) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto range = ctx->cache.equal_range(g->hash);
    PlanEntry *pe = nullptr;
    for (auto it = range.first; it != range.second; ++it)
        if (it->second.geo->same_as(*g)) {
            pe = &it->second;
            break;
        }
    if (!pe) {
        auto it = ctx->cache.emplace(g->hash, PlanEntry{g, {}});
        pe = &it->second;
    }
    if (canon) *canon = pe->geo;
    if (layout) {
        if (!pe->layout) pe->layout = std::make_shared<const SiteLayout>(build_site_layout(*pe->geo));
        *layout = pe->layout;
    }
    const int key = K | (full ? 1 << 8 : 0);  // K <= 32
    auto f = pe->plans.find(key);
    if (f != pe->plans.end()) return f->second;
    auto p = build_plan(*pe->geo, K, err, full);
    if (p) pe->plans[key] = p;
    return p;
}

size_t align256(size_t x);

// Host contents of a plan's instance tables (see PlanTables): the records of
// every class instance, instance-major per class, and every instance's
// weight offset; tab_off / iw_off give each class's first entry.
struct PlanTablesHost {
    std::vector<InstStep> tab;
    std::vector<int32_t> iw;
    std::vector<size_t> tab_off, iw_off;
    PlanTables pt;  // per-class counts and kinds (device pointers unset)
};

void plan_tables_host(const GeoPlan *p, const Geometry &g, PlanTablesHost *h) {
    std::vector<int64_t> soff(g.n_sites + 1, 0);
    for (int s2 = 0; s2 < g.n_sites; ++s2) {
        int64_t sz = 1;
        for (int l = 0; l < g.rank[s2]; ++l) sz *= g.dim[g.slot(s2, l)];
        soff[s2 + 1] = soff[s2] + sz;
    }
    auto stride_of = [&](int site, int slot) {
        int64_t st2 = 1;
        for (int l = g.rank[site] - 1; l > slot; --l) st2 *= g.dim[g.slot(site, l)];
        return st2;
    };
    const int ncls = (int)p->classes.size();
    std::vector<InstStep> &tab = h->tab;
    std::vector<int32_t> &iw = h->iw;
    std::vector<size_t> &tab_off = h->tab_off, &iw_off = h->iw_off;
    tab_off.assign(ncls, 0);
    iw_off.assign(ncls, 0);
    PlanTables &pt = h->pt;
    pt.cls.resize(ncls);
    for (int c = 0; c < ncls; ++c) {
        const ClassDesc &cd = p->classes[c];
        PlanTables::Cls &pc = pt.cls[c];
        tab_off[c] = tab.size();
        iw_off[c] = iw.size();
        pc.n_inst = (int)p->inst_cluster[c].size();
        pc.wide_stride = 0;
        pc.scalar = (cd.max_f == 1 && cd.out_size == 1) ? 1 : 0;
        const std::vector<int> &cyc = p->loop_order[c];
        pc.loop_e = 0;
        if (!pc.scalar && !cyc.empty() && p->loop_e[c] >= 2 && p->loop_e[c] <= 5 && (int)cyc.size() == 3 * cd.n_verts)
            pc.loop_e = p->loop_e[c];
        for (int k = 0; k < pc.n_inst; ++k) {
            iw.push_back((int32_t)p->w_off[p->inst_cluster[c][k]]);
            if (pc.loop_e) {
                for (int j = 0; j < cd.n_verts; ++j) {
                    const int v = cyc[3 * j];
                    const int site = p->inst_site[c][(size_t)k * cd.n_verts + v];
                    const uint32_t slots = p->inst_slots[c][(size_t)k * cd.n_verts + v];
                    InstStep r;
                    std::memset(&r, 0, sizeof r);
                    const int64_t s_in = stride_of(site, (int)((slots >> (4 * cyc[3 * j + 1])) & 15u));
                    const int64_t s_out = stride_of(site, (int)((slots >> (4 * cyc[3 * j + 2])) & 15u));
                    r.xs[0] = (int32_t)s_in;
                    r.xs[1] = (int32_t)s_out;
                    r.xoff = (int32_t)(soff[site] + s_in + s_out);  // excited indices start at 1
                    tab.push_back(r);
                }
                continue;
            }
            for (int st2 = 0; st2 < cd.n_steps; ++st2) {
                const StepDesc &sd = p->steps[cd.step_begin + st2];
                const int site = p->inst_site[c][(size_t)k * cd.n_verts + sd.vert];
                const uint32_t slots = p->inst_slots[c][(size_t)k * cd.n_verts + sd.vert];
                InstStep r;
                std::memset(&r, 0, sizeof r);
                int64_t xo = soff[site];
                for (int m = 0; m < sd.n_xl; ++m) {
                    const int64_t sm = stride_of(site, (int)((slots >> (4 * m)) & 15u));
                    r.xs[m] = (int32_t)sm;
                    if (sm >= (int64_t(1) << 24)) pc.wide_stride = 1;
                    if (sd.x_excited[m]) xo += sm;  // excited indices start at 1
                }
                r.xoff = (int32_t)xo;
                tab.push_back(r);
            }
        }
    }
}

// The plan's device instance tables (see PlanTables), built on its first use
// with g its geometry; the upload is complete on return.
// nullptr (with *st set) when the device memory cannot be had.
const PlanTables *plan_tables(pne_ctx *ctx, const GeoPlan *p, const Geometry &g, pne_status *st) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->plan_tables.find(p);
    if (it != ctx->plan_tables.end()) return &it->second;
    PlanTablesHost h;
    plan_tables_host(p, g, &h);
    const std::vector<InstStep> &tab = h.tab;
    const std::vector<int32_t> &iw = h.iw;
    PlanTables pt = h.pt;
    const int ncls = (int)p->classes.size();
    const size_t tab_bytes = align256(std::max<size_t>(1, tab.size()) * sizeof(InstStep));
    pt.bytes = tab_bytes + align256(std::max<size_t>(1, iw.size()) * sizeof(int32_t));
    if (ctx->budget && ctx->used + pt.bytes > ctx->budget) {
        *st = fail(ctx, PNE_ERR_OUT_OF_MEMORY, "memory budget exceeded (cluster tables)");
        return nullptr;
    }
    if (hipMalloc(&pt.dev, pt.bytes) != hipSuccess) {
        *st = fail(ctx, PNE_ERR_OUT_OF_MEMORY, "device allocation failed (cluster tables)");
        return nullptr;
    }
    hipError_t e = hipSuccess;
    if (!tab.empty())
        e = hipMemcpyAsync(pt.dev, tab.data(), tab.size() * sizeof(InstStep), hipMemcpyHostToDevice, ctx->up_stream);
    if (e == hipSuccess && !iw.empty())
        e = hipMemcpyAsync((char *)pt.dev + tab_bytes, iw.data(), iw.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->up_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->up_stream);  // any stream may use the tables next
    if (e != hipSuccess) {
        (void)hipFree(pt.dev);
        *st = hip_fail(ctx, e, "cluster table upload");
        return nullptr;
    }
    for (int c = 0; c < ncls; ++c) {
        pt.cls[c].tab = (const InstStep *)pt.dev + h.tab_off[c];
        pt.cls[c].iw = (const int32_t *)((const char *)pt.dev + tab_bytes) + h.iw_off[c];
    }
    ctx->used += pt.bytes;
    return &ctx->plan_tables.emplace(p, std::move(pt)).first->second;
}

// Device memory of a batch: every table and buffer is a 256-byte aligned
// piece of one allocation.  Tables with host contents come first, so one
// copy from the context's pinned staging buffer uploads all of them.
struct ArenaPlan {
    struct Piece {
        const void *src;  // host contents, or nullptr for a device-only buffer
        size_t bytes;
        void **dst;
        size_t off;
    };
    std::vector<Piece> up, buf;
    template <class T>
    void upload(const std::vector<T> &v, const T **dst) {
        if (v.empty()) {
            *dst = nullptr;
            return;
        }
        up.push_back({v.data(), v.size() * sizeof(T), (void **)dst, 0});
    }
    template <class T>
    void buffer(size_t bytes, T **dst) {
        buf.push_back({nullptr, bytes ? bytes : 8, (void **)dst, 0});
    }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Lay the pieces out, place them (a new allocation, or the batch's fixed
// region when `fixed` is set), let `fixup` patch host contents that hold
// device addresses of other pieces, then upload the host contents.
pne_status commit_arena(pne_batch *b, ArenaPlan &ap, const StaticArena *fixed,
                        const std::function<void()> &fixup) {
    pne_ctx *ctx = b->ctx;
    size_t off = 0;
    for (auto &pc : ap.up) {
        pc.off = off;
        off += align256(pc.bytes);
    }
    const size_t up_bytes = off;
    for (auto &pc : ap.buf) {
        pc.off = off;
        off += align256(pc.bytes);
    }
    const size_t total = off;
    void *p = nullptr;
    if (fixed) {
        if (total > fixed->cap)
            return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "batch needs " + std::to_string(total) +
                                                        " bytes, more than the fixed scratch region holds (" +
                                                        std::to_string(fixed->cap) + ")");
        p = fixed->base;
    } else {
        if (ctx->budget && ctx->used + total > ctx->budget)
            return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "memory budget exceeded");
        if (hipMalloc(&p, total) != hipSuccess) return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "device allocation failed");
        b->allocs.push_back(p);
        b->bytes += total;
        ctx->used += total;
    }
    for (auto &pc : ap.up) *pc.dst = (char *)p + pc.off;
    for (auto &pc : ap.buf) *pc.dst = (char *)p + pc.off;
    if (fixup) fixup();
    if (!up_bytes) return PNE_OK;
    if (fixed) {
        // pageable staging on the batch stream, complete before returning
        std::vector<char> st(up_bytes);
        for (auto &pc : ap.up) std::memcpy(st.data() + pc.off, pc.src, pc.bytes);
        hipError_t e = hipMemcpyAsync(p, st.data(), up_bytes, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "table upload");
        return PNE_OK;
    }
    if (ctx->up_pending) {  // the previous upload still reads the staging buffer
        hipError_t e = hipEventSynchronize(ctx->up_done);
        if (e != hipSuccess) return hip_fail(ctx, e, "upload wait");
        ctx->up_pending = false;
    }
    if (ctx->staging_bytes < up_bytes) {
        if (ctx->staging) (void)hipHostFree(ctx->staging);
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        const size_t want = std::max(up_bytes + up_bytes / 2, (size_t)1 << 20);
        if (hipHostMalloc(&ctx->staging, want, hipHostMallocDefault) != hipSuccess)
            return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "pinned allocation failed");
        ctx->staging_bytes = want;
    }
    char *st = (char *)ctx->staging;
    for (auto &pc : ap.up) std::memcpy(st + pc.off, pc.src, pc.bytes);
    hipError_t e = hipMemcpyAsync(p, st, up_bytes, hipMemcpyHostToDevice, ctx->up_stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->up_done, ctx->up_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ctx->up_done, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "table upload");
    ctx->up_pending = true;
    return PNE_OK;
}

// h_state from the last waited launch's pinned slot (once per wait)
void ensure_state(pne_batch *b) {
    if (b->state_slot < 0) return;
    const NetState *src = b->h_state_slot[b->state_slot];
    b->h_state.assign(src, src + b->nets.size());
    b->state_slot = -1;
}

hipError_t enqueue_result_copies(pne_batch *b) {
    const int n = (int)b->nets.size();
    hipError_t e = hipMemcpyAsync(b->h_results_pinned, b->db.results, sizeof(NetResult) * n, hipMemcpyDeviceToHost,
                                  b->stream);
    if (e != hipSuccess) return e;
    if (b->open_total > 0) {
        const int slot = (int)(b->h_results_pinned == b->h_results_slot[1]);
        e = hipMemcpyAsync(b->h_open_slot[slot], b->db.open_out, sizeof(double) * b->open_total,
                           hipMemcpyDeviceToHost, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipMemcpyAsync(b->h_state_pinned, b->db.state, sizeof(NetState) * n, hipMemcpyDeviceToHost, b->stream);
}

// The launch sequence of a batch without per-launch BP networks (what a
// graph capture records; the result copies follow it outside the graph,
// into the launch's pinned slot).
hipError_t enqueue_all(pne_batch *b) {
    const DeviceBatch &db = b->db;
    hipStream_t s = b->stream;
    hipError_t e;
    if ((e = launch_init(db, s)) != hipSuccess) return e;
    if ((e = launch_fused(db, b->opt.bp_tol, b->opt.bp_max_iter, s)) != hipSuccess) return e;
    if ((e = launch_regauge(db, s)) != hipSuccess) return e;
    if ((e = launch_clusters(db, s)) != hipSuccess) return e;
    return launch_combine(db, s);
}

hipEvent_t take_event(pne_batch *b) {
    if (!b->ev_pool.empty()) {
        hipEvent_t e = b->ev_pool.back();
        b->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Launch `fn` on the batch stream, bracketed by events when profiling.
template <class F>
hipError_t timed(pne_batch *b, int kid, F &&fn) {
    // launchers with nothing to do enqueue nothing, and are not timed either
    const DeviceBatch &db = b->db;
    const bool work = kid == KID_INIT ? (db.n_init_sites > 0 || db.n_init_nets > 0)
                    : kid == KID_FUSED ? db.n_fused > 0
                    : kid == KID_REGAUGE ? (db.n_rg_tiles > 0 || db.n_rg_wide > 0 || db.n_rg_sites > 0)
                    : kid == KID_CLUSTERS ? db.n_cblocks > 0
                    : kid == KID_COMBINE ? db.n_combine > 0
                    : true;
    const bool prof = work && (b->opt.flags & PNE_FLAG_PROFILE) != 0 &&
                      (b->opt.profile_kernels == 0 || ((b->opt.profile_kernels >> kid) & 1));
    hipStream_t s = b->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
        e0 = take_event(b);
        e1 = take_event(b);
        hipError_t e = hipEventRecord(e0, s);
        if (e != hipSuccess) return e;
    }
    hipError_t err = fn(s);
    if (err != hipSuccess) return err;
    if (prof) {
        err = hipEventRecord(e1, s);
        b->ev_used.push_back({b->n_launched, kid, e0, e1});
    }
    return err;
}

// Fold in the kernel times of launches up to `upto` (exclusive), which have
// completed; events of a still outstanding launch stay for its own wait.
void collect_times(pne_batch *b, int64_t upto) {
    std::vector<pne_batch::TimedLaunch> keep;
    for (auto &u : b->ev_used) {
        if (u.launch >= upto) {
            keep.push_back(u);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, u.e0, u.e1) == hipSuccess) {
            b->kt_ms[u.kid] += ms;
            b->kt_n[u.kid] += 1;
        }
        b->ev_pool.push_back(u.e0);
        b->ev_pool.push_back(u.e1);
    }
    b->ev_used.swap(keep);
}

void free_batch(pne_batch *b) {
    for (auto &u : b->ev_used) {
        (void)hipEventDestroy(u.e0);
        (void)hipEventDestroy(u.e1);
    }
    b->ev_used.clear();
    for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
    b->ev_pool.clear();
    for (void *p : b->allocs) (void)hipFree(p);
    b->allocs.clear();
    for (hipEvent_t &e : b->done_slot) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    for (hipEvent_t *e : {&b->db.fork, &b->db.join}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
    b->db.side = nullptr;
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
    if (b->h_pinned) (void)hipHostFree(b->h_pinned);
    b->h_pinned = nullptr;
    b->h_state_pinned = nullptr;
    b->h_results_pinned = nullptr;
    if (b->ctx) b->ctx->used -= std::min(b->ctx->used, b->bytes);
}

}  // namespace

extern "C" {

pne_status pne_options_default(pne_options *opt) {
    if (!opt) return PNE_ERR_INVALID_ARG;
    std::memset(opt, 0, sizeof *opt);
    opt->max_excited = 4;
    opt->precision = PNE_FP64;
    opt->bp_tol = 1e-13;
    opt->bp_max_iter = 500;
    opt->bp_check_every = 0;
    opt->mode = PNE_MODE_LOOP;
    opt->bp_damping = 0.0;
    opt->err_bound = 1e-5;
    return PNE_OK;
}

const char *pne_last_error(const pne_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    return g_tls_err.c_str();
}

pne_status pne_ctx_create(int device, size_t budget, void *stream, pne_ctx **out) {
    if (!out) return fail(nullptr, PNE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(nullptr, PNE_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(nullptr, PNE_ERR_INVALID_ARG, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, PNE_ERR_DEVICE, "hipSetDevice failed");
    auto *c = new pne_ctx();
    c->device = device;
    c->budget = budget;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->wall_khz = khz;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, PNE_ERR_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->up_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->up_done, hipEventDisableTiming) != hipSuccess) {
        if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
        if (c->up_stream) (void)hipStreamDestroy(c->up_stream);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return fail(nullptr, PNE_ERR_DEVICE, "upload stream creation failed");
    }
    *out = c;
    return PNE_OK;
}

pne_status pne_ctx_destroy(pne_ctx *ctx) {
    if (!ctx) return PNE_ERR_INVALID_ARG;
    if (ctx->up_stream) (void)hipStreamSynchronize(ctx->up_stream);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->up_done) (void)hipEventDestroy(ctx->up_done);
    if (ctx->up_stream) (void)hipStreamDestroy(ctx->up_stream);
    if (ctx->side_stream) {
        (void)hipStreamSynchronize(ctx->side_stream);
        (void)hipStreamDestroy(ctx->side_stream);
    }
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    for (auto &kv : ctx->plan_tables) (void)hipFree(kv.second.dev);
    delete ctx;
    return PNE_OK;
}

pne_status pne_network_create(pne_ctx *ctx, const pne_network_desc *desc, int on_device, pne_network **out) {
    return ctx ? pne::network_create_on(ctx, desc, on_device, ctx->stream, out) : PNE_ERR_INVALID_ARG;
}

}  // extern "C"

int pne::network_sites(pne_network *net) { return net->geo->n_sites; }
bool pne::network_graph(pne_network *net, std::vector<int> *rank, std::vector<int> *bond_dims, std::vector<int> *bu,
                        std::vector<int> *bul, std::vector<int> *bv, std::vector<int> *bvl) {
    const Geometry &g = *net->geo;
    if (g.n_open > 0) return false;
    *rank = g.rank;
    *bu = g.bu;
    *bul = g.bul;
    *bv = g.bv;
    *bvl = g.bvl;
    bond_dims->clear();
    for (int b = 0; b < g.n_bonds; ++b) bond_dims->push_back(g.dim[g.slot(g.bu[b], g.bul[b])]);
    return true;
}
const double *pne::network_site_ptr(pne_network *net, int site) { return net->dptr[site]; }
bool pne::same_geometry(pne_network *a, pne_network *b) { return a->geo->same_as(*b->geo); }
hipStream_t pne::ctx_stream(pne_ctx *ctx) { return ctx->stream; }
double *pne::ctx_rank_times(pne_ctx *ctx) { return ctx->rank_ms; }
int pne::ctx_device(pne_ctx *ctx) { return ctx->device; }
pne_status pne::ctx_fail(pne_ctx *ctx, pne_status st, const std::string &msg) { return fail(ctx, st, msg); }

pne_status pne::network_create_on(pne_ctx *ctx, const pne_network_desc *desc, int on_device, hipStream_t stream,
                                  pne_network **out) {
    if (!ctx || !desc || !out) return fail(ctx, PNE_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto g = std::make_shared<Geometry>();
    std::string why = build_geometry(desc, g.get());
    if (!why.empty()) return fail(ctx, PNE_ERR_INVALID_ARG, why);
    if (!desc->site_data) return fail(ctx, PNE_ERR_INVALID_ARG, "site_data is NULL");
    for (int s = 0; s < g->n_sites; ++s)
        if (!desc->site_data[s]) return fail(ctx, PNE_ERR_INVALID_ARG, "site tensor pointer is NULL");
    auto *net = new pne_network();
    net->ctx = ctx;
    net->geo = g;
    net->dptr.resize(g->n_sites);
    std::vector<size_t> sz(g->n_sites);
    size_t total = 0;
    for (int s = 0; s < g->n_sites; ++s) {
        size_t n = 1;
        for (int l = 0; l < g->rank[s]; ++l) n *= (size_t)g->dim[g->slot(s, l)];
        sz[s] = n;
        total += n;
    }
    if (on_device) {
        for (int s = 0; s < g->n_sites; ++s) net->dptr[s] = desc->site_data[s];
    } else {
        // reject non-finite inputs before they reach the device
        for (int s = 0; s < g->n_sites; ++s)
            for (size_t i = 0; i < sz[s]; ++i)
                if (!std::isfinite(desc->site_data[s][i])) {
                    delete net;
                    return fail(ctx, PNE_ERR_INVALID_ARG, "non-finite tensor entry");
                }
        size_t bytes = total * sizeof(double);
        if (ctx->budget && ctx->used + bytes > ctx->budget) {
            delete net;
            return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "memory budget exceeded");
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            delete net;
            return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "device allocation failed");
        }
        net->owned = (double *)p;
        net->owned_bytes = bytes;
        ctx->used += bytes;
        std::vector<double> host(total);
        size_t off = 0;
        for (int s = 0; s < g->n_sites; ++s) {
            std::memcpy(host.data() + off, desc->site_data[s], sz[s] * sizeof(double));
            net->dptr[s] = net->owned + off;
            off += sz[s];
        }
        hipError_t e = hipMemcpyAsync(p, host.data(), bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            (void)hipFree(p);
            ctx->used -= bytes;
            delete net;
            return hip_fail(ctx, e, "tensor upload");
        }
    }
    *out = net;
    return PNE_OK;
}

extern "C" {


pne_status pne_network_set_partitions(pne_network *net, int32_t n_partitions, const int32_t *part_begin,
                                      const int32_t *part_bond) {
    if (!net) return fail(nullptr, PNE_ERR_INVALID_ARG, "null network");
    // copy on write: batches made before keep the geometry they planned with
    auto g = std::make_shared<Geometry>(*net->geo);
    std::string why = set_partitions(g.get(), n_partitions, part_begin, part_bond);
    if (!why.empty())
        return fail(net->ctx, why.rfind("unsupported", 0) == 0 ? PNE_ERR_UNSUPPORTED : PNE_ERR_INVALID_ARG, why);
    net->geo = g;
    return PNE_OK;
}

pne_status pne_network_set_subpartitions(pne_network *net, uint32_t x_mask, int32_t n_sub, const int32_t *sub_begin,
                                         const int32_t *sub_bond) {
    if (!net) return fail(nullptr, PNE_ERR_INVALID_ARG, "null network");
    auto g = std::make_shared<Geometry>(*net->geo);
    std::string why = set_subpartitions(g.get(), x_mask, n_sub, sub_begin, sub_bond);
    if (!why.empty())
        return fail(net->ctx, why.rfind("unsupported", 0) == 0 ? PNE_ERR_UNSUPPORTED : PNE_ERR_INVALID_ARG, why);
    net->geo = g;
    return PNE_OK;
}

pne_status pne_network_destroy(pne_network *net) {
    if (!net) return PNE_ERR_INVALID_ARG;
    if (net->owned) {
        (void)hipFree(net->owned);
        net->ctx->used -= std::min(net->ctx->used, net->owned_bytes);
    }
    delete net;
    return PNE_OK;
}

pne_status pne_batch_create(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt,
                            pne_batch **out) {
    if (!ctx || !opt) return PNE_ERR_INVALID_ARG;
    if (opt->flags & PNE_FLAG_AUTOTUNE) {
        pne_options tuned;
        pne_status st = pne_autotune(ctx, nets, n, opt, 3, &tuned);
        if (st != PNE_OK) return st;
        return pne::batch_create_on(ctx, nets, n, &tuned, ctx->stream, out);
    }
    return pne::batch_create_on(ctx, nets, n, opt, ctx->stream, out);
}

// Signature of a batch for the tuning cache: the multiset of network
// geometries, K, the precision, the mode, the damping and the flags that
// change results.
static uint64_t batch_signature(pne_network *const *nets, int32_t n, const pne_options *opt) {
    std::vector<uint64_t> h(n);
    for (int i = 0; i < n; ++i) h[i] = nets[i]->geo->hash;
    std::sort(h.begin(), h.end());
    uint64_t x = 0x9e3779b97f4a7c15ull ^ (uint64_t)n;
    auto mix = [&](uint64_t v) {
        x ^= v + 0x9e3779b97f4a7c15ull + (x << 6) + (x >> 2);
    };
    for (uint64_t v : h) mix(v);
    mix((uint64_t)opt->max_excited);
    mix((uint64_t)opt->precision);
    mix((uint64_t)(opt->flags & (PNE_FLAG_NO_PERSISTENT | PNE_FLAG_BP_JACOBI)));
    mix((uint64_t)opt->mode);
    uint64_t damp_bits;
    std::memcpy(&damp_bits, &opt->bp_damping, sizeof damp_bits);
    mix(damp_bits);
    return x;
}

pne_status pne_autotune(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt, int32_t trials,
                        pne_options *best) {
    if (!ctx || !nets || n <= 0 || !opt || !best) return fail(ctx, PNE_ERR_INVALID_ARG, "bad autotune arguments");
    const uint32_t keep = opt->flags & ~(PNE_FLAG_AUTOTUNE | PNE_FLAG_GRAPH | PNE_FLAG_SEPARATE_REGAUGE);
    const uint64_t sig = batch_signature(nets, n, opt);
    auto apply = [&](const pne_ctx::Tuned &c) {
        *best = *opt;
        best->flags = keep | c.flags;
        best->small_sites = c.small_sites;
        best->tiles_in_flight = c.tiles_in_flight;
        best->reg_budget = c.reg_budget;
    };
    auto it = ctx->tuned.find(sig);
    if (it != ctx->tuned.end()) {
        apply(it->second);
        return PNE_OK;
    }
    if (trials < 1) trials = 1;
    // Candidates: the persistent kernel's tile shape (small-network block
    // threshold, tiles in flight, register budget) with eager launches, then
    // graph replay of the best of those.  The first candidate is the default.
    std::vector<pne_ctx::Tuned> cands;
    for (int rb : {0, 1})
        for (int ss : {0, 256})
            for (int nt : {0, 1, 2}) {
                pne_ctx::Tuned c;
                c.small_sites = ss;
                c.tiles_in_flight = nt;
                c.reg_budget = rb;
                cands.push_back(c);
            }
    auto time_variant = [&](const pne_ctx::Tuned &c, double *ms_out, bool *graphable) -> pne_status {
        pne_options o = *opt;
        o.flags = (keep & ~PNE_FLAG_PROFILE) | c.flags;
        o.small_sites = c.small_sites;
        o.tiles_in_flight = c.tiles_in_flight;
        o.reg_budget = c.reg_budget;
        pne_batch *b = nullptr;
        pne_status st = pne::batch_create_on(ctx, nets, n, &o, ctx->stream, &b);
        if (st != PNE_OK) return st;
        if (graphable) *graphable = b->db.n_tiles == 0;
        double ms = 1e300;
        for (int tr = 0; tr <= trials && st >= 0; ++tr) {  // the first run warms up
            const auto t0 = std::chrono::steady_clock::now();
            st = pne_batch_run(b, nullptr);
            const double dt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (tr > 0) ms = std::min(ms, dt);
        }
        pne_batch_destroy(b);
        *ms_out = ms;
        return st < 0 ? st : PNE_OK;
    };
    pne_ctx::Tuned bestc;
    double best_ms = 1e300, default_ms = 0.0;
    bool graphable = false;
    for (size_t k = 0; k < cands.size(); ++k) {
        double ms = 1e300;
        pne_status st = time_variant(cands[k], &ms, k == 0 ? &graphable : nullptr);
        if (st != PNE_OK) {
            if (k == 0) return st;  // the default variant must run
            continue;               // e.g. a variant whose LDS or register needs do not fit
        }
        if (k == 0) default_ms = ms;
        if (ms < best_ms) {
            best_ms = ms;
            bestc = cands[k];
        }
    }
    if (graphable) {
        pne_ctx::Tuned g = bestc;
        g.flags = PNE_FLAG_GRAPH;
        double ms = 1e300;
        if (time_variant(g, &ms, nullptr) == PNE_OK && ms < best_ms) {
            best_ms = ms;
            bestc = g;
        }
    }
    bestc.ms = best_ms;
    bestc.default_ms = default_ms;
    ctx->tuned[sig] = bestc;
    apply(bestc);
    return PNE_OK;
}

pne_status pne_tune_cache_save(pne_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(ctx, PNE_ERR_INVALID_ARG, "null argument");
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(ctx, PNE_ERR_INVALID_ARG, std::string("cannot write ") + tmp);
    std::fprintf(f, "{\"pne_tune_cache\": 1, \"entries\": [");
    bool first = true;
    for (const auto &kv : ctx->tuned) {
        const pne_ctx::Tuned &c = kv.second;
        std::fprintf(f,
                     "%s\n  {\"signature\": \"%016llx\", \"flags\": %u, \"small_sites\": %d, "
                     "\"tiles_in_flight\": %d, \"reg_budget\": %d, \"ms\": %.6g, \"default_ms\": %.6g}",
                     first ? "" : ",", (unsigned long long)kv.first, c.flags, c.small_sites, c.tiles_in_flight,
                     c.reg_budget, c.ms, c.default_ms);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0 && std::rename(tmp.c_str(), path) == 0;
    return ok ? PNE_OK : fail(ctx, PNE_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

pne_status pne_tune_cache_load(pne_ctx *ctx, const char *path, int32_t *n_loaded) {
    if (!ctx || !path) return fail(ctx, PNE_ERR_INVALID_ARG, "null argument");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(ctx, PNE_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::string s;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, got);
    std::fclose(f);
    if (s.find("\"pne_tune_cache\"") == std::string::npos)
        return fail(ctx, PNE_ERR_INVALID_ARG, "not a tuning cache file");
    // every entry is one {...} object with the keys written by pne_tune_cache_save
    auto field = [](const std::string &obj, const char *key, double *out) {
        const std::string k = std::string("\"") + key + "\":";
        const size_t p = obj.find(k);
        if (p == std::string::npos) return false;
        char *end = nullptr;
        *out = std::strtod(obj.c_str() + p + k.size(), &end);
        return end != obj.c_str() + p + k.size();
    };
    int32_t cnt = 0;
    size_t pos = s.find('[');
    while (pos != std::string::npos) {
        const size_t a = s.find('{', pos), e = a == std::string::npos ? a : s.find('}', a);
        if (a == std::string::npos || e == std::string::npos) break;
        const std::string obj = s.substr(a, e - a + 1);
        pos = e + 1;
        const size_t sp = obj.find("\"signature\":");
        if (sp == std::string::npos) return fail(ctx, PNE_ERR_INVALID_ARG, "tuning cache entry without a signature");
        const size_t q = obj.find('"', sp + 12);
        const uint64_t sig = std::strtoull(obj.c_str() + q + 1, nullptr, 16);
        double v[6];
        const char *keys[6] = {"flags", "small_sites", "tiles_in_flight", "reg_budget", "ms", "default_ms"};
        for (int k = 0; k < 6; ++k)
            if (!field(obj, keys[k], &v[k])) return fail(ctx, PNE_ERR_INVALID_ARG, "malformed tuning cache entry");
        pne_ctx::Tuned c;
        c.flags = (uint32_t)v[0] & (PNE_FLAG_GRAPH | PNE_FLAG_SEPARATE_REGAUGE);
        c.small_sites = (int32_t)v[1];
        c.tiles_in_flight = (int32_t)v[2];
        c.reg_budget = (int32_t)v[3];
        c.ms = v[4];
        c.default_ms = v[5];
        if (c.small_sites < 0 || c.tiles_in_flight < 0 || c.tiles_in_flight > 2 || c.reg_budget < 0 ||
            c.reg_budget > 1)
            return fail(ctx, PNE_ERR_INVALID_ARG, "tuning cache entry out of range");
        ctx->tuned[sig] = c;
        ++cnt;
    }
    if (n_loaded) *n_loaded = cnt;
    return PNE_OK;
}

}  // extern "C"

pne_status pne::batch_create_on(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt,
                                hipStream_t stream, pne_batch **out, const StaticArena *fixed) {
    if (!ctx || !nets || n <= 0 || !opt || !out) return fail(ctx, PNE_ERR_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    if (opt->max_excited < 0 || opt->max_excited > 32) return fail(ctx, PNE_ERR_INVALID_ARG, "K must be in [0, 32]");
    if (opt->precision < 0 || opt->precision > 2) return fail(ctx, PNE_ERR_INVALID_ARG, "unknown precision");
    if (!(opt->bp_tol >= 0.0) || opt->bp_max_iter < 1) return fail(ctx, PNE_ERR_INVALID_ARG, "bad BP options");
    if (opt->mode < PNE_MODE_LOOP || opt->mode > PNE_MODE_CUMULANT) return fail(ctx, PNE_ERR_INVALID_ARG, "unknown mode");
    if (!(opt->bp_damping >= 0.0 && opt->bp_damping < 1.0))
        return fail(ctx, PNE_ERR_INVALID_ARG, "bp_damping must be in [0, 1)");
    if (!(opt->err_bound >= 0.0)) return fail(ctx, PNE_ERR_INVALID_ARG, "err_bound must be >= 0");
    if (opt->small_sites < 0 || opt->tiles_in_flight < 0 || opt->tiles_in_flight > 2 || opt->reg_budget < 0 ||
        opt->reg_budget > 1)
        return fail(ctx, PNE_ERR_INVALID_ARG, "bad tile options");
    if (fixed && (opt->flags & (PNE_FLAG_PROFILE | PNE_FLAG_GRAPH | PNE_FLAG_AUTOTUNE)))
        return fail(ctx, PNE_ERR_INVALID_ARG, "profiling, graph replay and autotuning allocate: not available here");
    for (int i = 0; i < n; ++i)
        if (!nets[i] || nets[i]->ctx != ctx) return fail(ctx, PNE_ERR_INVALID_ARG, "network from another context");

    auto b = std::make_unique<pne_batch>();
    b->ctx = ctx;
    b->stream = stream;
    b->fixed = fixed != nullptr;
    b->nets.assign(nets, nets + n);
    b->opt = *opt;
    const int K = opt->max_excited;
    const int prec = opt->precision;
    const size_t esz = prec == PNE_FP64 ? 8 : prec == PNE_FP32 ? 4 : 2;

    // plans, and each geometry's site layout
    std::vector<std::shared_ptr<const SiteLayout>> layouts;
    layouts.reserve(n);
    for (int i = 0; i < n; ++i) {
        std::string err;
        std::shared_ptr<Geometry> canon;
        std::shared_ptr<const SiteLayout> lay;
        auto p = get_plan(ctx, nets[i]->geo, K, opt->mode == PNE_MODE_FULL, &err, &canon, &lay);
        if (!p) {
            bool unsup = err.rfind("unsupported", 0) == 0;
            return fail(ctx, unsup ? PNE_ERR_UNSUPPORTED : PNE_ERR_INVALID_ARG, err);
        }
        if ((int)p->buckets.size() > 64) return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: too many term buckets");
        if (opt->mode == PNE_MODE_CUMULANT) {
            if (p->open_a >= 0 || p->listed)
                return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: the cumulant form takes closed networks without partitions");
            if (!p->csize.empty() && 3 * *std::min_element(p->csize.begin(), p->csize.end()) <= K)
                return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: the second-order cumulant form needs K < 3 x the smallest cluster");
        }
        b->plans.push_back(p);
        layouts.push_back(std::move(lay));
    }

    // sites, messages, transforms, slices
    std::vector<SiteRec> sites;
    std::vector<int> net_of_site;
    {
        size_t total_sites = 0;
        for (int i = 0; i < n; ++i) total_sites += (size_t)nets[i]->geo->n_sites;
        sites.reserve(total_sites);
        net_of_site.reserve(total_sites);
    }
    int64_t msg = 0, sl = 0, vac = 0;
    b->site_base.resize(n);
    for (int i = 0; i < n; ++i) {
        const Geometry &g = *nets[i]->geo;
        b->site_base[i] = (int)sites.size();
        for (int s = 0; s < g.n_sites; ++s) {
            SiteRec r;
            std::memset(&r, 0, sizeof r);
            r.t = nets[i]->dptr[s];
            r.net = i;
            r.rank = g.rank[s];
            r.msg_off = (int)msg;
            r.slice_off = sl;
            r.vac_off = -1;
            int size = 1, mo = 0, omask = 0, nopen = 1;
            for (int l = r.rank - 1; l >= 0; --l) {
                r.stride[l] = size;
                size *= g.dim[g.slot(s, l)];
            }
            for (int l = 0; l < r.rank; ++l) {
                int d = g.dim[g.slot(s, l)];
                r.dim[l] = d;
                r.moff[l] = mo;
                mo += d;
                if (g.is_open[g.slot(s, l)]) {
                    omask |= 1 << l;
                    nopen *= d;
                }
            }
            r.size = size;
            r.open_mask = omask;
            if (omask) {
                r.vac_off = (int)vac;
                vac += nopen;
            }
            msg += mo;
            sl += size;
            sites.push_back(r);
            net_of_site.push_back(i);
        }
    }
    if (msg > INT32_MAX) return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: batch too large");
    // partner destinations
    for (int i = 0; i < n; ++i) {
        const Geometry &g = *nets[i]->geo;
        int base = b->site_base[i];
        for (int s = 0; s < g.n_sites; ++s) {
            SiteRec &r = sites[base + s];
            for (int l = 0; l < r.rank; ++l) {
                const int p = g.partner[g.slot(s, l)];
                const int ps = layouts[i]->slot_site[p];
                const int pl = p - g.slot_base[ps];
                r.dst[l] = sites[base + ps].msg_off + sites[base + ps].moff[pl];
            }
        }
        for (int bb = 0; bb < g.n_bonds; ++bb) sites[base + g.bv[bb]].vside_mask |= 1 << g.bvl[bb];
    }
    b->msg_total = msg;

    // BP tiles: per network, runs of sites with identical leg dims.  A network
    // whose tiles all take the register path and whose messages fit in LDS is
    // run by the persistent BP kernel; the others are swept launch by launch.
    std::vector<BpTile> tiles;
    std::vector<int> tile_sites;
    std::vector<FusedNet> fused;
    std::vector<FusedGroup> fgroups;
    std::vector<int> fsite_list;
    // per-launch sweep tiles in three launches, each with its own dynamic LDS:
    // register tiles, LDS tiles, register tiles of the wide shapes
    std::vector<BpTile> reg_tiles, lds_tiles, wide_tiles, xwide_tiles;
    std::vector<size_t> tile_need;  // dynamic LDS bytes of each entry of tiles
    size_t reg_lds = 0, wide_lds = 0, xwide_lds = 0;
    const size_t bp_budget = 16 * 1024 / 8;  // doubles of dynamic LDS per tile (several waves per CU)
    // doubles of dynamic LDS per persistent block: two blocks per CU, or one
    // with the 256-VGPR kernel
    const size_t fused_budget = (opt->reg_budget ? 155 : 79) * 1024 / 8;
    // networks over that budget but within the 256-VGPR kernel's run in it,
    // one block per CU, in a launch of their own
    const size_t big_budget = 155 * 1024 / 8;
    std::vector<char> fused_big;  // per fused entry
    const int small_sites = opt->small_sites > 0 ? opt->small_sites : kPSmallSites;
    auto tiles_for = [&](int dim, int rank) {
        return (opt->tiles_in_flight > 0 && bp_persistent_tiles_tunable(dim, rank)) ? opt->tiles_in_flight
                                                                                     : bp_persistent_tiles_in_flight(dim, rank);
    };
    size_t bp_lds = 0;
    std::vector<char> net_rg_inline(n, 0);  // gauge + slices built by the persistent block
    std::vector<char> net_fused(n, 0);      // BP in a persistent block
    std::vector<int> fused_of_net(n, -1);   // index of the network's persistent block
    for (int i = 0; i < n; ++i) {
        const Geometry &g = *nets[i]->geo;
        int base = b->site_base[i];
        const SiteLayout &lay = *layouts[i];
        bool first_tile_of_net = true;
        const int tile_begin = (int)tiles.size();
        bool all_reg = g.n_open == 0;
        for (auto &kv : lay.groups) {
            const SiteRec &r0 = sites[base + kv.second[0]];
            int nos = 0;
            for (int l = 0; l < r0.rank; ++l) nos += r0.dim[l];
            const int last = r0.dim[r0.rank - 1];
            int maxd = 1;
            for (int l = 0; l < r0.rank; ++l) maxd = std::max(maxd, r0.dim[l]);
            // per-site share of the tile's LDS (the reduction scratch is shared)
            const size_t per = 3 * (size_t)nos + (size_t)r0.size + 2 * (size_t)(r0.size / last);
            const int rows0 = r0.size / last;
            int cap = (int)std::max<size_t>(1, std::min<size_t>(64, bp_budget / per));
            cap = std::min(cap, std::max(1, bp_tile_threads() / std::max(rows0, nos)));
            int dc = maxd;
            for (int l = 0; l < r0.rank; ++l)
                if (r0.dim[l] != maxd) dc = 0;
            if (dc < 2 || dc > 6) dc = 0;
            const int reg_spt = dc ? bp_sweep_reg_sites_per_tile(dc, r0.rank) : 0;
            if (reg_spt > 0) cap = reg_spt;
            if (!(dc && bp_reg_sites_per_tile(dc, r0.rank) > 0)) all_reg = false;  // persistent tiles
            if (!reg_spt && per > 150 * 1024 / 8)
                return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: site tensor too large for LDS");
            for (size_t k = 0; k < kv.second.size(); k += cap) {
                BpTile t;
                std::memset(&t, 0, sizeof t);
                t.site_begin = (int)tile_sites.size();
                t.n_sites = (int)std::min<size_t>(cap, kv.second.size() - k);
                t.net = i;
                t.rank = r0.rank;
                t.size = r0.size;
                t.n_os = nos;
                t.first = first_tile_of_net ? 1 : 0;
                t.dc = dc;
                t.reg = reg_spt > 0 ? 1 : 0;
                first_tile_of_net = false;
                for (int j = 0; j < t.n_sites; ++j) tile_sites.push_back(base + kv.second[k + j]);
                const size_t need = t.reg ? (size_t)t.n_sites * nos * 8
                                          : bp_tile_lds_doubles(t.n_sites, r0.size, nos, last, maxd) * 8;
                tiles.push_back(t);
                tile_need.push_back(need);
            }
        }
        // persistent path: every shape group on the register path, LDS fits
        int64_t msg_lo = sites[base].msg_off;
        int64_t msg_hi = sites[base + g.n_sites - 1].msg_off;
        {
            const SiteRec &rl = sites[base + g.n_sites - 1];
            for (int l = 0; l < rl.rank; ++l) msg_hi += rl.dim[l];
        }
        const int msg_size = (int)(msg_hi - msg_lo);
        int pscratch = 0;
        for (auto &kv : lay.groups) {
            const SiteRec &r0 = sites[base + kv.second[0]];
            const int spw = bp_persistent_sites_per_tile(r0.dim[0], r0.rank);
            if (spw > 0)
                pscratch = std::max(pscratch, bp_persistent_scratch(spw, r0.rank, r0.dim[0], tiles_for(r0.dim[0], r0.rank)));
        }
        // two-colouring of the site graph for the red-black schedule
        const std::vector<int> &colour = lay.colour;
        const bool bip = !(opt->flags & PNE_FLAG_BP_JACOBI) && lay.bipartite;
        // gauge + slices inside the persistent block when every shape has a
        // register-path regauge; its per-wave transform table shares the scratch
        // (dropped again when the larger scratch would not fit the LDS budget)
        bool rg_inline = !(opt->flags & PNE_FLAG_SEPARATE_REGAUGE);
        int rg_scratch = pscratch;
        for (auto &kv : lay.groups) {
            const SiteRec &r0 = sites[base + kv.second[0]];
            if (!bp_persistent_regauge_supported(r0.dim[0], r0.rank)) {
                rg_inline = false;
                break;
            }
            rg_scratch = std::max(rg_scratch, bp_persistent_regauge_table(r0.dim[0], r0.rank));
        }
        // the in-block term sum needs 153 doubles of the waves' scratch (8 x 32, or 2 x 80 in the
        // two-wave blocks of small networks)
        const bool small = g.n_sites <= small_sites;
        rg_scratch = std::max(rg_scratch, small ? 80 : 32);
        // the budget of the network's launch: the batch's, or the 256-VGPR
        // kernel's for a large network that does not fit the batch's
        size_t budget = fused_budget;
        if (!small && fused_budget < big_budget &&
            bp_persistent_lds_doubles(msg_size, g.n_sites, pscratch, bip ? 1 : 2, small) > fused_budget)
            budget = big_budget;
        if (rg_inline && bp_persistent_lds_doubles(msg_size, g.n_sites, rg_scratch, bip ? 1 : 2, small) <= budget)
            pscratch = rg_scratch;
        else
            rg_inline = false;
        const size_t pneed = bp_persistent_lds_doubles(msg_size, g.n_sites, pscratch, bip ? 1 : 2, small);
        // damped BP runs launch by launch (Jacobi, the damped mix in the per-launch normalisation)
        if (all_reg && pneed <= budget && !(opt->flags & PNE_FLAG_NO_PERSISTENT) && opt->bp_damping == 0.0) {
            fused_big.push_back(pneed > fused_budget ? 1 : 0);
            FusedNet f;
            std::memset(&f, 0, sizeof f);
            f.net = i;
            f.msg_base = (int)msg_lo;
            f.msg_size = msg_size;
            f.site_base = base;
            f.n_sites = g.n_sites;
            f.group_begin = (int)fgroups.size();
            f.list_begin = (int)fsite_list.size();
            f.scratch = pscratch;
            f.colors = bip ? 2 : 1;
            f.rg_inline = rg_inline ? 1 : 0;
            net_rg_inline[i] = rg_inline ? 1 : 0;
            for (int c = 0; c < f.colors; ++c)
                for (auto &kv : lay.groups) {
                    const SiteRec &r0 = sites[base + kv.second[0]];
                    FusedGroup fg;
                    std::memset(&fg, 0, sizeof fg);
                    fg.dc = r0.dim[0];
                    fg.rank = r0.rank;
                    fg.spw = bp_persistent_sites_per_tile(fg.dc, fg.rank);
                    fg.nt = tiles_for(fg.dc, fg.rank);
                    fg.color = c;
                    fg.list_off = (int)fsite_list.size() - f.list_begin;
                    for (int ls : kv.second)
                        if (!bip || colour[ls] == c) fsite_list.push_back(ls);
                    fg.n_sites = (int)fsite_list.size() - f.list_begin - fg.list_off;
                    if (fg.n_sites > 0) fgroups.push_back(fg);
                }
            f.n_groups = (int)fgroups.size() - f.group_begin;
            fused_of_net[i] = (int)fused.size();
            fused.push_back(f);
            net_fused[i] = 1;
        } else {
            for (size_t t = tile_begin; t < tiles.size(); ++t) {
                const BpTile &tt = tiles[t];
                if (tt.reg && bp_sweep_xwide(tt.dc, tt.rank)) {
                    xwide_tiles.push_back(tt);
                    xwide_lds = std::max(xwide_lds, tile_need[t]);
                } else if (tt.reg && bp_reg_sites_per_tile(tt.dc, tt.rank) == 0) {
                    wide_tiles.push_back(tt);
                    wide_lds = std::max(wide_lds, tile_need[t]);
                } else if (tt.reg) {
                    reg_tiles.push_back(tt);
                    reg_lds = std::max(reg_lds, tile_need[t]);
                } else {
                    lds_tiles.push_back(tt);
                    bp_lds = std::max(bp_lds, tile_need[t]);
                }
            }
        }
    }

    // cluster tables: classes shared per distinct plan, instances per class
    std::vector<ClassDesc> classes;
    std::vector<StepDesc> steps;
    std::vector<StepEnt> step_ents;
    std::vector<ClusterBlock> cblocks;
    std::vector<PlanNet> pnets;
    std::vector<CombineRec> crec(n);
    std::vector<GeoRec> geos;
    std::vector<Bucket> buckets;
    std::vector<int> pair_a, pair_b;
    std::vector<PairCat> pair_cats;
    std::vector<int> coll_off, coll_cl;
    std::vector<double> coll_coef;
    std::map<const GeoPlan *, int> plan_index;  // -> first class id
    std::map<const GeoPlan *, int> geo_index;
    int64_t wtot = 0;
    b->w_base.resize(n);
    b->open_off.assign(n, -1);
    size_t cl_lds = 0;
    for (int i = 0; i < n; ++i) {
        const GeoPlan *p = b->plans[i].get();
        b->w_base[i] = wtot;
        wtot += p->w_total;
        if (!plan_index.count(p)) {
            plan_index[p] = (int)classes.size();
            for (const ClassDesc &cd0 : p->classes) {
                ClassDesc cd = cd0;
                cd.step_begin += (int)steps.size();
                const size_t asz = prec == PNE_FP64 ? 8 : 4;
                // per instance slot: F and G, then the step's summed-entry offsets
                const size_t slots = (size_t)(256 / cd.group);
                const size_t fg = slots * 2 * (size_t)cd.max_f * asz;
                if (fg + slots * (size_t)cd.max_sum * sizeof(StepEnt) > 64 * 1024) cd.max_sum = 0;
                classes.push_back(cd);
                cl_lds = std::max(cl_lds, fg + slots * (size_t)cd.max_sum * sizeof(StepEnt));
            }
            const int ent_base = (int)step_ents.size();
            for (StepDesc sd : p->steps) {
                if (sd.ent >= 0) sd.ent += ent_base;
                steps.push_back(sd);
            }
            step_ents.insert(step_ents.end(), p->step_ents.begin(), p->step_ents.end());
            GeoRec gr;
            std::memset(&gr, 0, sizeof gr);
            gr.K = K;
            gr.n_buckets = (int)p->buckets.size();
            gr.bucket_begin = (int)buckets.size();
            buckets.insert(buckets.end(), p->buckets.begin(), p->buckets.end());
            gr.pair_begin = (int)pair_a.size();
            gr.n_pairs = (int)p->pair_a.size();
            pair_a.insert(pair_a.end(), p->pair_a.begin(), p->pair_a.end());
            pair_b.insert(pair_b.end(), p->pair_b.begin(), p->pair_b.end());
            gr.pair_cat_begin = (int)pair_cats.size();
            gr.n_pair_cats = (int)p->pair_cats.size();
            pair_cats.insert(pair_cats.end(), p->pair_cats.begin(), p->pair_cats.end());
            if (p->listed) {
                gr.listed = 1;
                gr.coll_begin = (int)coll_off.size();
                gr.n_colls = (int)p->coll_off.size() - 1;
                gr.coll_cl_begin = (int)coll_cl.size();
                coll_off.insert(coll_off.end(), p->coll_off.begin(), p->coll_off.end());
                coll_cl.insert(coll_cl.end(), p->coll_cl.begin(), p->coll_cl.end());
                gr.coef_begin = -1;
                if (!p->coll_coef.empty()) {
                    gr.coef_begin = (int)coll_coef.size();
                    coll_coef.insert(coll_coef.end(), p->coll_coef.begin(), p->coll_coef.end());
                }
                if (coll_cl.size() > (size_t)INT32_MAX / 2)
                    return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: too many listed configurations");
            }
            geo_index[p] = (int)geos.size();
            geos.push_back(gr);
        }
        CombineRec &cr = crec[i];
        std::memset(&cr, 0, sizeof cr);
        cr.w_base = b->w_base[i];
        cr.n_clusters = p->clusters.count();
        cr.geo = geo_index[p];
        cr.site_begin = b->site_base[i];
        cr.n_sites = nets[i]->geo->n_sites;
        cr.vac_a = p->open_a >= 0 ? sites[b->site_base[i] + p->open_a].vac_off : -1;
        cr.vac_b = p->open_b >= 0 ? sites[b->site_base[i] + p->open_b].vac_off : -1;
        cr.pa = p->pa;
        cr.pb = p->pb;
        cr.open_off = -1;
        cr.cumulant = opt->mode == PNE_MODE_CUMULANT ? 1 : 0;
        if (p->open_a >= 0) {
            cr.open_off = (int32_t)b->open_total;
            b->open_total += (int64_t)p->pa * p->pb;
        }
        b->open_off[i] = cr.open_off;
    }
    if (cl_lds > 64 * 1024) return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: cluster frontier too large for LDS");
    // Classes point at their plan's device instance tables (kept by the
    // context); a network only adds its slice and weight bases.  Blocks walk
    // the plan's networks in order, each block covering up to 256/group
    // consecutive (network, instance) pairs of one class.
    std::vector<char> net_cl_fused(n, 0);
    const bool cl_separate = (opt->flags & PNE_FLAG_SEPARATE_REGAUGE) != 0;
    // fixed region: per plan, the host instance tables and their device addresses
    struct FixedPlanTables {
        PlanTablesHost h;
        int class_begin = 0;
        const InstStep *tab_dev = nullptr;
        const int32_t *iw_dev = nullptr;
    };
    std::deque<FixedPlanTables> fixed_tables;
    {
        std::map<const GeoPlan *, std::vector<int>> nets_of_plan;
        std::vector<const GeoPlan *> plan_order;
        for (int i = 0; i < n; ++i) {
            const GeoPlan *p = b->plans[i].get();
            if (!nets_of_plan.count(p)) plan_order.push_back(p);
            nets_of_plan[p].push_back(i);
        }
        for (const GeoPlan *p : plan_order) {
            const std::vector<int> &pn_all = nets_of_plan[p];
            const Geometry &g = *nets[pn_all[0]]->geo;
            const int c0 = plan_index[p];
            const int ncls = (int)p->classes.size();
            pne_status pst = PNE_OK;
            const PlanTables *pt = nullptr;
            if (fixed) {
                // the instance tables go into the batch's own region (uploaded
                // with the other tables; class pointers patched at commit)
                fixed_tables.emplace_back();
                FixedPlanTables &ft = fixed_tables.back();
                plan_tables_host(p, g, &ft.h);
                ft.class_begin = c0;
                pt = &ft.h.pt;
            } else {
                pt = plan_tables(ctx, p, g, &pst);
            }
            if (!pt) return pst;
            // A closed network whose BP, gauge and slices run in a persistent
            // block, and whose plan has only scalar and cycle classes, also
            // gets its clusters and term sum from that block.
            bool plan_fast = g.n_open == 0 && !cl_separate && !p->listed;
            for (int c = 0; c < ncls && plan_fast; ++c) {
                const ClassDesc &cd = classes[c0 + c];
                const bool sc = cd.max_f == 1 && cd.out_size == 1;
                const bool lp = !p->loop_order[c].empty() && p->loop_e[c] >= 2 && p->loop_e[c] <= 5;
                plan_fast = sc || lp;
            }
            std::vector<int> pn;  // networks left to the cluster and combine launches
            for (int i : pn_all) {
                if (plan_fast && net_fused[i] && net_rg_inline[i]) {
                    FusedNet &f = fused[fused_of_net[i]];
                    f.cl_fused = 1;
                    f.class_begin = c0;
                    f.n_classes = ncls;
                    f.w_base = b->w_base[i];
                    net_cl_fused[i] = 1;
                } else {
                    pn.push_back(i);
                }
            }
            const int pnet_begin = (int)pnets.size();
            for (int i : pn) pnets.push_back(PlanNet{sites[b->site_base[i]].slice_off, b->w_base[i], i, 0});
            for (int c = 0; c < ncls; ++c) {
                ClassDesc &cd = classes[c0 + c];
                const PlanTables::Cls &pc = pt->cls[c];
                cd.tab = pc.tab;
                cd.iw = pc.iw;
                cd.n_inst = pc.n_inst;
                cd.pnet_begin = pnet_begin;
                cd.n_pnets = (int)pn.size();
                cd.scalar = pc.scalar;
                cd.loop_e = pc.loop_e;
                if (pc.wide_stride) cd.max_sum = 0;
            }
            // blocks: networks in order, classes interleaved
            std::vector<int> pend_begin(ncls, 0), pend_count(ncls, 0);
            auto emit = [&](int c) {
                ClusterBlock cb;
                cb.cls = c0 + c;
                cb.flat_begin = pend_begin[c];
                cb.count = pend_count[c];
                cb.pad = 0;
                cblocks.push_back(cb);
                pend_count[c] = 0;
            };
            for (size_t j = 0; j < pn.size(); ++j)
                for (int c = 0; c < ncls; ++c) {
                    const ClassDesc &cd = classes[c0 + c];
                    const int ipb = (cd.scalar || cd.loop_e) ? 256 : 256 / cd.group;
                    int64_t f0 = (int64_t)j * cd.n_inst, f1 = f0 + cd.n_inst;
                    while (f0 < f1) {
                        if (pend_count[c] == 0) pend_begin[c] = (int)f0;
                        const int64_t take = std::min<int64_t>(ipb - pend_count[c], f1 - f0);
                        pend_count[c] += (int)take;
                        f0 += take;
                        if (pend_count[c] == ipb) emit(c);
                    }
                }
            for (int c = 0; c < ncls; ++c)
                if (pend_count[c] > 0) emit(c);
        }
        if (pnets.size() > (size_t)INT32_MAX)
            return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: batch too large");
    }

    // device allocation
    size_t regauge_lds = 0;
    for (const SiteRec &r : sites) regauge_lds = std::max(regauge_lds, regauge_site_lds_doubles(r) * 8);
    if (regauge_lds > 150 * 1024) return fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: site tensor too large for LDS");
    pne_status st;
    DeviceBatch &db = b->db;
    ArenaPlan ap;
#define UP(vec, field) ap.upload(vec, &db.field)
    UP(sites, sites);
    const int n_reg = (int)reg_tiles.size();
    std::vector<BpTile> loop_tiles(std::move(reg_tiles));
    loop_tiles.insert(loop_tiles.end(), lds_tiles.begin(), lds_tiles.end());
    const int n_narrow = (int)loop_tiles.size();
    loop_tiles.insert(loop_tiles.end(), wide_tiles.begin(), wide_tiles.end());
    const int n_wide_end = (int)loop_tiles.size();
    loop_tiles.insert(loop_tiles.end(), xwide_tiles.begin(), xwide_tiles.end());
    UP(loop_tiles, tiles);
    UP(tiles, all_tiles);
    // Wave priority by work per BP step (tensor entries): where blocks of light
    // and heavy networks share a CU, the heavy ones get the issue slots first,
    // so both finish closer together and the heavy ones leave a shorter tail.
    if (!fused.empty()) {
        std::vector<int64_t> work(fused.size());
        for (size_t k = 0; k < fused.size(); ++k) {
            int64_t wk = 0;
            for (int s2 = 0; s2 < fused[k].n_sites; ++s2) wk += sites[fused[k].site_base + s2].size;
            work[k] = wk;
        }
        std::vector<int64_t> sorted_work(work);
        std::sort(sorted_work.begin(), sorted_work.end());
        const int64_t light = sorted_work[sorted_work.size() / 4];  // lower quartile
        for (size_t k = 0; k < fused.size(); ++k) fused[k].prio = work[k] >= 2 * light ? 1 : 0;
    }
    // large networks first, then the small ones (their own launch, 128-thread
    // blocks), then the big ones (their own launch, the 256-VGPR kernel)
    {
        std::vector<int> order(fused.size());
        for (size_t k = 0; k < fused.size(); ++k) order[k] = (int)k;
        auto cls = [&](int k) { return fused_big[k] ? 2 : (fused[k].n_sites <= small_sites ? 1 : 0); };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls(x) < cls(y); });
        std::vector<FusedNet> sorted;
        std::vector<char> big_sorted;
        for (int k : order) {
            sorted.push_back(fused[k]);
            big_sorted.push_back(fused_big[k]);
        }
        fused.swap(sorted);
        fused_big.swap(big_sorted);
    }
    size_t lds_large = 0, lds_small = 0, lds_big = 0;
    int n_small = 0, n_big = 0;
    for (size_t k = 0; k < fused.size(); ++k) {
        const FusedNet &f = fused[k];
        const bool small = f.n_sites <= small_sites;
        const size_t need = bp_persistent_lds_doubles(f.msg_size, f.n_sites, f.scratch, f.colors == 2 ? 1 : 2, small) * 8;
        if (fused_big[k]) {
            lds_big = std::max(lds_big, need);
            ++n_big;
        } else if (small) {
            lds_small = std::max(lds_small, need);
            ++n_small;
        } else {
            lds_large = std::max(lds_large, need);
        }
    }
    UP(fused, fused);
    b->h_fused = fused;
    b->paths.assign(n, 0);
    for (int i = 0; i < n; ++i)
        b->paths[i] = (net_fused[i] ? PNE_PATH_PERSISTENT : 0) | (net_rg_inline[i] ? PNE_PATH_BLOCK_GAUGE : 0) |
                      (net_cl_fused[i] ? PNE_PATH_BLOCK_TERMS : 0);
    UP(fgroups, fgroups);
    UP(fsite_list, fsite_list);
    // regauge work: register tiles without open legs, other sites one per block
    std::vector<int> rg_tiles, rg_wide, rg_sites;
    for (size_t t = 0; t < tiles.size(); ++t) {
        if (net_rg_inline[tiles[t].net]) continue;
        bool open = false;
        for (int j = 0; j < tiles[t].n_sites; ++j) open = open || sites[tile_sites[tiles[t].site_begin + j]].open_mask;
        if (tiles[t].reg && !open && regauge_reg_supported(tiles[t].dc, tiles[t].rank)) {
            rg_tiles.push_back((int)t);
        } else if (tiles[t].reg && !open && tiles[t].n_sites <= regauge_wide_sites(tiles[t].dc, tiles[t].rank)) {
            rg_wide.push_back((int)t);
        } else {
            for (int j = 0; j < tiles[t].n_sites; ++j) rg_sites.push_back(tile_sites[tiles[t].site_begin + j]);
        }
    }
    // the wide-shape regauge, one launch per shape (regauge_wide_supported lists
    // kRgWideShapes shapes, so the groups fit)
    std::stable_sort(rg_wide.begin(), rg_wide.end(), [&](int x, int y) {
        return tiles[x].dc * 8 + tiles[x].rank < tiles[y].dc * 8 + tiles[y].rank;
    });
    db.n_rg_wide_groups = 0;
    for (size_t g0 = 0; g0 < rg_wide.size();) {
        const int key = tiles[rg_wide[g0]].dc * 8 + tiles[rg_wide[g0]].rank;
        size_t g1 = g0;
        while (g1 < rg_wide.size() && tiles[rg_wide[g1]].dc * 8 + tiles[rg_wide[g1]].rank == key) ++g1;
        db.rg_wide_shape[db.n_rg_wide_groups] = key;
        db.rg_wide_begin[db.n_rg_wide_groups++] = (int)g0;
        g0 = g1;
    }
    db.rg_wide_begin[db.n_rg_wide_groups] = (int)rg_wide.size();
    // the per-site regauge in size groups (each up to twice its smallest
    // site; the last takes the rest), launched with their own LDS
    std::stable_sort(rg_sites.begin(), rg_sites.end(),
                     [&](int x, int y) { return regauge_site_lds_doubles(sites[x]) < regauge_site_lds_doubles(sites[y]); });
    db.n_rg_groups = 0;
    for (size_t g0 = 0; g0 < rg_sites.size();) {
        const int gi = db.n_rg_groups++;
        const size_t lo = regauge_site_lds_doubles(sites[rg_sites[g0]]);
        size_t g1 = g0, hi = lo;
        while (g1 < rg_sites.size() &&
               (gi == DeviceBatch::kRgGroups - 1 || regauge_site_lds_doubles(sites[rg_sites[g1]]) <= 2 * lo)) {
            hi = std::max(hi, regauge_site_lds_doubles(sites[rg_sites[g1]]));
            ++g1;
        }
        db.rg_group_begin[gi] = (int)g0;
        db.rg_group_lds[gi] = hi * 8;
        g0 = g1;
    }
    db.rg_group_begin[db.n_rg_groups] = (int)rg_sites.size();
    UP(rg_tiles, rg_tiles);
    UP(rg_wide, rg_wide);
    UP(rg_sites, rg_sites);
    db.n_rg_tiles = (int)rg_tiles.size();
    db.n_rg_wide = (int)rg_wide.size();
    db.n_rg_sites = (int)rg_sites.size();
    UP(tile_sites, tile_sites);
    // k_init resets the messages of networks swept launch by launch only
    std::vector<int> init_sites;
    for (int i = 0; i < n; ++i)
        if (!net_fused[i])
            for (int s2 = 0; s2 < nets[i]->geo->n_sites; ++s2) init_sites.push_back(b->site_base[i] + s2);
    UP(init_sites, init_sites);
    db.n_init_sites = (int)init_sites.size();
    std::vector<int> init_nets;
    for (int i = 0; i < n; ++i)
        if (!net_fused[i]) init_nets.push_back(i);
    UP(init_nets, init_nets);
    db.n_init_nets = (int)init_nets.size();
    UP(classes, classes);
    UP(steps, steps);
    UP(step_ents, step_ents);
    db.n_step_ents = (int)step_ents.size();
    // blocks by kernel path (frontier plans; cycles of leg dimension 2, 3, 4,
    // 5; scalar products), each launched with the registers of its own
    // path; order kept within a path
    constexpr int kClKinds = DeviceBatch::kClKinds;
    int cl_kind_begin[kClKinds + 1] = {};
    {
        auto kind = [&](const ClusterBlock &cb) {
            const ClassDesc &cd = classes[cb.cls];
            return cd.scalar ? kClKinds - 1 : (cd.loop_e ? cd.loop_e - 1 : 0);
        };
        std::vector<ClusterBlock> sorted;
        sorted.reserve(cblocks.size());
        for (int k = 0; k < kClKinds; ++k) {
            cl_kind_begin[k] = (int)sorted.size();
            for (const ClusterBlock &cb : cblocks)
                if (kind(cb) == k) sorted.push_back(cb);
        }
        cl_kind_begin[kClKinds] = (int)sorted.size();
        cblocks.swap(sorted);
    }
    UP(cblocks, cblocks);
    UP(pnets, pnets);
    UP(crec, crec);
    std::vector<int> combine_nets;  // networks whose terms the combine launch sums
    for (int i = 0; i < n; ++i)
        if (!net_cl_fused[i]) combine_nets.push_back(i);
    UP(combine_nets, combine_nets);
    db.n_combine = (int)combine_nets.size();
    UP(geos, geos);
    UP(buckets, buckets);
    UP(pair_a, pair_a);
    UP(pair_b, pair_b);
    UP(pair_cats, pair_cats);
    UP(coll_off, coll_off);
    UP(coll_cl, coll_cl);
    UP(coll_coef, coll_coef);
    for (FixedPlanTables &ft : fixed_tables) {
        ap.upload(ft.h.tab, &ft.tab_dev);
        ap.upload(ft.h.iw, &ft.iw_dev);
    }
#undef UP
    db.n_sites = (int)sites.size();
    db.n_tiles = (int)loop_tiles.size();
    db.n_narrow_tiles = n_narrow;
    db.n_reg_tiles = n_reg;
    db.reg_lds = reg_lds;
    db.wide_lds = wide_lds;
    db.xwide_lds = xwide_lds;
    db.n_wide_end = n_wide_end;
    db.n_fused = (int)fused.size();
    db.fused_lds = lds_large;
    db.fused_lds_small = lds_small;
    db.n_fused_small = n_small;
    db.fused_lds_big = lds_big;
    db.n_fused_big = n_big;
    db.n_nets = n;
    db.n_cblocks = (int)cblocks.size();
    for (int k = 0; k <= kClKinds; ++k) db.cl_kind_begin[k] = cl_kind_begin[k];
    db.bp_lds = bp_lds;
    db.regauge_lds = regauge_lds;
    db.cluster_lds = cl_lds;
    db.precision = prec;
    db.damping = opt->bp_damping;
    db.bp_stall = opt->bp_stall_steps == 0 ? 50 : std::max(0, opt->bp_stall_steps);
    db.bp_floor = 100.0 * opt->bp_tol;
    db.reg_budget = opt->reg_budget;
#define AL(bytes, field, type) ap.buffer((bytes), &db.field)
    AL(sizeof(NetState) * n, state, NetState *);
    AL(sizeof(double) * msg, msg0, double *);
    AL(sizeof(double) * msg, msg1, double *);
    AL(esz * std::max<int64_t>(sl, 1), slices, void *);
    db.n_slice_elems = sl;
    db.n_w = wtot;
    AL(sizeof(double) * sites.size(), site_log, double *);
    AL(sizeof(int) * sites.size(), site_sign, int *);
    AL(sizeof(double) * std::max<int64_t>(vac, 1), vac, double *);
    AL(sizeof(double) * std::max<int64_t>(wtot, 1), w, double *);
    AL(sizeof(NetResult) * n, results, NetResult *);
    AL(sizeof(double) * std::max<int64_t>(b->open_total, 1), open_out, double *);
#undef AL
    // classes of plans whose instance tables sit in the fixed region point at
    // them once the region's layout is known (before the upload copies them)
    auto fixup = [&]() {
        for (FixedPlanTables &ft : fixed_tables)
            for (size_t c = 0; c < ft.h.pt.cls.size(); ++c) {
                ClassDesc &cd = classes[ft.class_begin + c];
                cd.tab = ft.tab_dev ? ft.tab_dev + ft.h.tab_off[c] : nullptr;
                cd.iw = ft.iw_dev ? ft.iw_dev + ft.h.iw_off[c] : nullptr;
            }
    };
    st = commit_arena(b.get(), ap, fixed, fixup);
    if (st != PNE_OK) {
        free_batch(b.get());
        return st;
    }
    // one pinned block for the per-network state and results read back by every wait
    const size_t st_bytes = align256(sizeof(NetState) * n);
    const size_t res_bytes = align256(sizeof(NetResult) * n);
    const size_t slot_bytes = st_bytes + res_bytes + align256(sizeof(double) * std::max<int64_t>(b->open_total, 1));
    char *slots = nullptr;
    if (fixed) {
        b->h_host.assign(2 * slot_bytes + 256, 0);  // pageable; copies complete at the stream synchronisation
        slots = b->h_host.data() + (256 - (reinterpret_cast<uintptr_t>(b->h_host.data()) & 255)) % 256;
    } else {
        if (hipHostMalloc(&b->h_pinned, 2 * slot_bytes, hipHostMallocDefault) != hipSuccess) {
            free_batch(b.get());
            return fail(ctx, PNE_ERR_OUT_OF_MEMORY, "pinned allocation failed");
        }
        slots = (char *)b->h_pinned;
    }
    for (int k = 0; k < 2; ++k) {
        b->h_state_slot[k] = (NetState *)(slots + k * slot_bytes);
        b->h_results_slot[k] = (NetResult *)(slots + k * slot_bytes + st_bytes);
        b->h_open_slot[k] = (double *)(slots + k * slot_bytes + st_bytes + res_bytes);
        if (fixed) continue;
        if (hipEventCreateWithFlags(&b->done_slot[k], hipEventDisableTiming) != hipSuccess) {
            free_batch(b.get());
            return fail(ctx, PNE_ERR_DEVICE, "event creation failed");
        }
    }
    // sweeps with wide and other tiles run the others on the side stream
    if (!fixed && b->db.n_narrow_tiles > 0 && b->db.n_tiles > b->db.n_narrow_tiles) {
        if (hipEventCreateWithFlags(&b->db.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->db.join, hipEventDisableTiming) != hipSuccess) {
            free_batch(b.get());
            return fail(ctx, PNE_ERR_DEVICE, "event creation failed");
        }
        b->db.side = ctx->side_stream;
    }
    b->h_state_pinned = b->h_state_slot[0];
    b->h_results_pinned = b->h_results_slot[0];
    b->msg_off.resize(sites.size());
    for (size_t s = 0; s < sites.size(); ++s) b->msg_off[s] = sites[s].msg_off;
    *out = b.release();
    return PNE_OK;
}

extern "C" {


pne_status pne_batch_launch(pne_batch *b) {
    if (!b) return PNE_ERR_INVALID_ARG;
    pne_ctx *ctx = b->ctx;
    hipStream_t s = b->stream;
    const DeviceBatch &db = b->db;
    if (b->n_launched - b->n_waited >= (b->fixed ? 1 : 2))
        return fail(ctx, PNE_ERR_INVALID_ARG, "too many launches outstanding");
    const int slot = (int)(b->n_launched & 1);
    if (b->state_slot == slot) ensure_state(b);  // this launch rewrites that slot
    b->h_state_pinned = b->h_state_slot[slot];
    b->h_results_pinned = b->h_results_slot[slot];
    // Graph replay: a batch whose BP runs entirely in persistent blocks has
    // no host decision inside a run, so its whole sequence (kernels and the
    // result copies) is captured once and replayed.
    if ((b->opt.flags & PNE_FLAG_GRAPH) && !(b->opt.flags & PNE_FLAG_PROFILE) && db.n_tiles == 0 && s != nullptr) {
        if (!b->graph_exec) {
            HIP_TRY(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_all(b);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(ctx, e != hipSuccess ? e : e2, "graph capture");
            }
            b->graph = g;
            HIP_TRY(ctx, hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
        }
        HIP_TRY(ctx, hipGraphLaunch(b->graph_exec, s));
        HIP_TRY(ctx, enqueue_result_copies(b));
        HIP_TRY(ctx, hipEventRecord(b->done_slot[slot], s));
        ++b->n_launched;
        b->launched = true;
        b->waited = false;
        return PNE_OK;
    }
    HIP_TRY(ctx, timed(b, KID_INIT, [&](hipStream_t st) { return launch_init(db, st); }));
    const int max_iter = b->opt.bp_max_iter;
    const double tol = b->opt.bp_tol;
    HIP_TRY(ctx, timed(b, KID_FUSED, [&](hipStream_t st) { return launch_fused(db, tol, max_iter, st); }));
    // Networks not run by the persistent kernel are swept one launch per
    // sweep, in chunks; after each chunk the host reads the per-network state
    // and stops once every network has stopped, failed, or reached the
    // tolerance on the chunk's last sweep.
    const int n = db.n_nets;
    int sweep = 0;
    int chunk = b->opt.bp_check_every > 0 ? b->opt.bp_check_every : b->first_chunk;
    // residual of each running network at the previous check: with the
    // current one it gives the network's geometric rate, and from that the
    // sweeps it still needs, so the next chunk ends near the last network's
    // convergence instead of a fixed doubling past it
    std::vector<double> prev_r(db.n_tiles > 0 ? n : 0, -1.0);
    int prev_last = -1;
    while (db.n_tiles > 0 && sweep < max_iter) {
        const int kk = std::min(chunk, max_iter - sweep);
        for (int j = 0; j < kk; ++j, ++sweep)
            HIP_TRY(ctx, timed(b, KID_SWEEP, [&](hipStream_t st) { return launch_sweep(db, sweep, tol, max_iter, st); }));
        HIP_TRY(ctx, hipMemcpyAsync(b->h_state_pinned, db.state, sizeof(NetState) * n, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        const int last = sweep - 1;
        bool all_done = true;
        int need = 0;  // largest predicted remaining sweeps (0: no running network has a rate yet)
        for (int i = 0; i < n; ++i) {
            const NetState &st = b->h_state_pinned[i];
            if (st.stop >= 0 || st.status < 0) continue;
            const double r = [&] {
                double d;
                std::memcpy(&d, &st.res_acc[last % 3], sizeof d);
                return d;
            }();
            if (r <= tol) continue;
            all_done = false;
            if (prev_last >= 0 && prev_r[i] > 0.0 && r > 0.0 && r < prev_r[i]) {
                const double lq = std::log(r / prev_r[i]) / (double)(last - prev_last);  // log rate per sweep
                const double left = std::log(tol / r) / lq;
                if (std::isfinite(left)) need = std::max(need, (int)std::ceil(left));
            }
            prev_r[i] = r;
        }
        prev_last = last;
        if (all_done) break;
        if (b->opt.bp_check_every <= 0)
            chunk = need > 0 ? std::min(need + 1, 32) : std::min(chunk * 2, 16);
    }
    // the close kernel finishes per-launch networks only (persistent blocks
    // record their own final state)
    if (db.n_tiles > 0)
        HIP_TRY(ctx, timed(b, KID_CLOSE, [&](hipStream_t st) { return launch_close(db, sweep - 1, tol, st); }));
    HIP_TRY(ctx, timed(b, KID_REGAUGE, [&](hipStream_t st) { return launch_regauge(db, st); }));
    HIP_TRY(ctx, timed(b, KID_CLUSTERS, [&](hipStream_t st) { return launch_clusters(db, st); }));
    HIP_TRY(ctx, timed(b, KID_COMBINE, [&](hipStream_t st) { return launch_combine(db, st); }));
    // results and state go to pinned memory in the same stream order, so the
    // host can enqueue further work (another batch) before waiting on this one
    HIP_TRY(ctx, enqueue_result_copies(b));
    if (b->done_slot[slot]) HIP_TRY(ctx, hipEventRecord(b->done_slot[slot], s));
    ++b->n_launched;
    b->launched = true;
    b->waited = false;
    return PNE_OK;
}

pne_status pne_batch_wait(pne_batch *b, pne_result *results) {
    if (!b || b->n_waited >= b->n_launched)
        return fail(b ? b->ctx : nullptr, PNE_ERR_INVALID_ARG, "batch not launched");
    pne_ctx *ctx = b->ctx;
    const int n = (int)b->nets.size();
    const int slot = (int)(b->n_waited & 1);
    if (b->done_slot[slot])
        HIP_TRY(ctx, hipEventSynchronize(b->done_slot[slot]));
    else
        HIP_TRY(ctx, hipStreamSynchronize(b->stream));
    ++b->n_waited;
    b->h_state_pinned = b->h_state_slot[slot];
    b->h_results_pinned = b->h_results_slot[slot];
    b->state_slot = slot;  // h_state is copied only if asked for
    collect_times(b, b->n_waited);
    b->waited = true;
    if (!results) return PNE_OK;
    pne_status worst = PNE_OK;
    for (int i = 0; i < n; ++i) {
        const NetResult &r = b->h_results_pinned[i];
        const NetState &s = b->h_state_pinned[i];
        const GeoPlan &p = *b->plans[i];
        pne_result &o = results[i];
        double *ov = o.open_values;
        int64_t cap = o.open_capacity;
        o.bp_iters = s.iters;
        o.bp_residual = s.residual;
        o.n_cluster_terms = p.clusters.count();
        o.n_config_terms = b->opt.mode == PNE_MODE_CUMULANT ? p.clusters.count() : p.n_configs;
        o.log_abs = r.log_abs;
        o.log_abs_bp = r.log_bp;
        o.sign = r.sign;
        o.n_open_values = 0;
        o.dangling_max = r.dangling;
        o.term_err_est = r.err_est;
        int st = s.status < 0 ? s.status : (s.converged ? PNE_OK : PNE_WARN_BP_NOT_CONVERGED);
        if (st >= 0 && !std::isfinite(r.log_abs)) st = PNE_ERR_SINGULAR;
        if (st == PNE_OK && b->opt.precision != PNE_FP64) {
            // closed: |delta ln|Z|| relative to max(1, |ln|Z||); open: relative entry error
            const double rel = p.open_a >= 0 ? r.err_est : r.err_est / std::max(1.0, std::fabs(r.log_abs));
            if (!(rel <= b->opt.err_bound)) st = PNE_WARN_PRECISION;
        }
        if (st >= 0 && p.open_a >= 0) {
            int m = p.pa * p.pb;
            if (!ov || cap < m) {
                st = PNE_ERR_INVALID_ARG;
            } else {
                const double *src = b->h_open_slot[slot] + b->open_off[i];
                for (int e = 0; e < m; ++e) ov[e] = src[e];
                o.n_open_values = m;
            }
        }
        o.status = st;
        if (st < 0 && (worst >= 0 || st < worst)) worst = (pne_status)st;
        else if (st > 0 && worst == PNE_OK) worst = (pne_status)st;
    }
    if (worst < 0) fail(ctx, worst, "one or more networks failed (see per-result status)");
    return worst;
}

pne_status pne_batch_run(pne_batch *b, pne_result *results) {
    pne_status s = pne_batch_launch(b);
    if (s != PNE_OK) return s;
    return pne_batch_wait(b, results);
}

pne_status pne_batch_destroy(pne_batch *b) {
    if (!b) return PNE_ERR_INVALID_ARG;
    if (b->ctx) (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
    return PNE_OK;
}

pne_status pne_contract_batch(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt,
                              pne_result *results) {
    pne_batch *b = nullptr;
    pne_status s = pne_batch_create(ctx, nets, n, opt, &b);
    if (s != PNE_OK) return s;
    s = pne_batch_run(b, results);
    pne_batch_destroy(b);
    return s;
}

pne_status pne_contract(pne_ctx *ctx, pne_network *net, const pne_options *opt, pne_result *res) {
    return pne_contract_batch(ctx, &net, 1, opt, res);
}

pne_status pne_enumerate_clusters(const pne_network_desc *desc, int32_t K, int64_t *n_clusters, int64_t *n_entries,
                                  int32_t *sizes, int32_t *bonds) {
    if (!desc || !n_clusters || !n_entries) return fail(nullptr, PNE_ERR_INVALID_ARG, "null argument");
    Geometry g;
    std::string why = build_geometry(desc, &g);
    if (!why.empty()) return fail(nullptr, PNE_ERR_INVALID_ARG, why);
    std::string err;
    auto p = build_plan(g, K, &err);
    if (!p) return fail(nullptr, err.rfind("unsupported", 0) == 0 ? PNE_ERR_UNSUPPORTED : PNE_ERR_INVALID_ARG, err);
    const ClusterList &cl = p->clusters;
    if (bonds) {
        if (*n_clusters < cl.count() || *n_entries < (int64_t)cl.bonds.size())
            return fail(nullptr, PNE_ERR_INVALID_ARG, "output buffers too small");
        for (int c = 0; c < cl.count(); ++c) sizes[c] = cl.off[c + 1] - cl.off[c];
        std::memcpy(bonds, cl.bonds.data(), cl.bonds.size() * sizeof(int32_t));
    }
    *n_clusters = cl.count();
    *n_entries = (int64_t)cl.bonds.size();
    return PNE_OK;
}

pne_status pne_count_configurations(const pne_network_desc *desc, int32_t K, int32_t mode, int32_t n_partitions,
                                    const int32_t *part_begin, const int32_t *part_bond, int64_t *n_clusters,
                                    int64_t *n_configs) {
    if (!desc || !n_clusters || !n_configs) return fail(nullptr, PNE_ERR_INVALID_ARG, "null argument");
    if (K < 0 || K > 32) return fail(nullptr, PNE_ERR_INVALID_ARG, "K must be in [0, 32]");
    if (mode != PNE_MODE_LOOP && mode != PNE_MODE_FULL) return fail(nullptr, PNE_ERR_INVALID_ARG, "unknown mode");
    Geometry g;
    std::string why = build_geometry(desc, &g);
    if (why.empty()) why = set_partitions(&g, n_partitions, part_begin, part_bond);
    if (!why.empty())
        return fail(nullptr, why.rfind("unsupported", 0) == 0 ? PNE_ERR_UNSUPPORTED : PNE_ERR_INVALID_ARG, why);
    std::string err;
    auto p = build_plan(g, K, &err, mode == PNE_MODE_FULL);
    if (!p) return fail(nullptr, err.rfind("unsupported", 0) == 0 ? PNE_ERR_UNSUPPORTED : PNE_ERR_INVALID_ARG, err);
    *n_clusters = p->clusters.count();
    *n_configs = p->n_configs;
    return PNE_OK;
}

pne_status pne_batch_kernel_times(pne_batch *b, double *ms_total, int64_t *launches, int32_t n, int32_t reset) {
    if (!b || !ms_total || !launches || n < 0) return fail(b ? b->ctx : nullptr, PNE_ERR_INVALID_ARG, "bad arguments");
    for (int k = 0; k < n; ++k) {
        ms_total[k] = k < KID_COUNT ? b->kt_ms[k] : 0.0;
        launches[k] = k < KID_COUNT ? b->kt_n[k] : 0;
    }
    if (reset)
        for (int k = 0; k < KID_COUNT; ++k) {
            b->kt_ms[k] = 0.0;
            b->kt_n[k] = 0;
        }
    return PNE_OK;
}

pne_status pne_batch_phase_times(pne_batch *b, double *out, int32_t n) {
    if (!b || !b->waited || !out || n < 0) return fail(b ? b->ctx : nullptr, PNE_ERR_INVALID_ARG, "bad arguments");
    double v[6] = {0, 0, 0, 0, 0, 0};
    unsigned long long t0 = ~0ull, t1 = 0, t2 = 0;
    int cnt = 0;
    const double tick_us = 1000.0 / b->ctx->wall_khz;
    ensure_state(b);
    for (const FusedNet &f : b->h_fused) {
        const NetState &s = b->h_state[f.net];
        if (s.t_bp < s.t_start || s.t_rg < s.t_bp) continue;
        const double bp = (double)(s.t_bp - s.t_start) * tick_us, rg = (double)(s.t_rg - s.t_bp) * tick_us;
        v[0] += bp;
        v[1] += rg;
        v[2] = std::max(v[2], bp);
        v[3] = std::max(v[3], rg);
        t0 = std::min(t0, s.t_start);
        t1 = std::max(t1, s.t_bp);
        t2 = std::max(t2, s.t_rg);
        ++cnt;
    }
    if (cnt) {
        v[0] /= cnt;
        v[1] /= cnt;
        v[4] = (double)(t1 - t0) * tick_us;
        v[5] = (double)(t2 - t0) * tick_us;
    }
    for (int k = 0; k < n; ++k) out[k] = k < 6 ? v[k] : 0.0;
    return PNE_OK;
}

pne_status pne_batch_paths(pne_batch *b, int32_t *out, int32_t n) {
    if (!b || !out || n != (int32_t)b->paths.size()) return fail(b ? b->ctx : nullptr, PNE_ERR_INVALID_ARG, "bad arguments");
    std::copy(b->paths.begin(), b->paths.end(), out);
    return PNE_OK;
}

pne_status pne_batch_messages(pne_batch *b, int32_t i, double *out, int64_t capacity) {
    if (!b || !b->waited || i < 0 || i >= (int)b->nets.size() || !out)
        return fail(b ? b->ctx : nullptr, PNE_ERR_INVALID_ARG, "bad arguments");
    const Geometry &g = *b->nets[i]->geo;
    int64_t need = 0;
    for (int bb = 0; bb < g.n_bonds; ++bb) need += 2 * g.dim[g.slot(g.bu[bb], g.bul[bb])];
    if (capacity < need) return fail(b->ctx, PNE_ERR_INVALID_ARG, "capacity too small");
    ensure_state(b);
    const double *src = b->h_state[i].parity ? b->db.msg1 : b->db.msg0;
    std::vector<double> host(b->msg_total);
    HIP_TRY(b->ctx, hipMemcpy(host.data(), src, sizeof(double) * b->msg_total, hipMemcpyDeviceToHost));
    int base = b->site_base[i];
    int64_t o = 0;
    for (int bb = 0; bb < g.n_bonds; ++bb) {
        int d = g.dim[g.slot(g.bu[bb], g.bul[bb])];
        int au = b->msg_off[base + g.bu[bb]];
        for (int l = 0; l < g.bul[bb]; ++l) au += g.dim[g.slot(g.bu[bb], l)];
        int cv = b->msg_off[base + g.bv[bb]];
        for (int l = 0; l < g.bvl[bb]; ++l) cv += g.dim[g.slot(g.bv[bb], l)];
        for (int k = 0; k < d; ++k) out[o++] = host[au + k];
        for (int k = 0; k < d; ++k) out[o++] = host[cv + k];
    }
    return PNE_OK;
}

pne_status pne_batch_cluster_weights(pne_batch *b, int32_t i, double *out, int64_t capacity, int64_t *n_values,
                                     int64_t *offsets) {
    if (!b || !b->waited || i < 0 || i >= (int)b->nets.size() || !n_values)
        return fail(b ? b->ctx : nullptr, PNE_ERR_INVALID_ARG, "bad arguments");
    const GeoPlan &p = *b->plans[i];
    *n_values = p.w_total;
    if (!out) return PNE_OK;
    if (capacity < p.w_total) return fail(b->ctx, PNE_ERR_INVALID_ARG, "capacity too small");
    if (p.w_total)
        HIP_TRY(b->ctx, hipMemcpy(out, b->db.w + b->w_base[i], sizeof(double) * p.w_total, hipMemcpyDeviceToHost));
    if (offsets)
        for (int c = 0; c < p.clusters.count(); ++c) offsets[c] = p.w_off[c];
    return PNE_OK;
}

}  // extern "C"
