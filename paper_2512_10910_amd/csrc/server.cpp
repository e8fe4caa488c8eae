// Request server: continuous batching of independent networks on one device.
//
// Clients submit networks from any thread (pne_submit copies the descriptor
// and the host tensors) and collect results with pne_poll (or learn which
// tickets finished from pne_server_completed).  Three threads own the
// context: the worker admits pending requests in arrival order while their
// estimated device bytes fit the memory budget, groups requests with
// identical options into one batch (plans are cached per lattice, so a batch
// of mixed lattices shares nothing but the launches), and keeps up to
// `pipeline_depth` batches being launched or in flight on separate streams,
// so the host work of the next batch (validation, uploads, tables) overlaps
// the device work of the current one; the launcher launches prepared batches
// in order (a batch whose networks sweep BP launch by launch waits on the
// device between sweep chunks); the completion thread hands a batch's
// results out as soon as the device has finished it.  A batch's networks
// stay resident from admission until its results are copied back.  Each
// network's result does not depend on which other networks share its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pne.h"
#include "runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t) {
    return std::chrono::duration<double>(t - t0).count();
}

struct Request {
    uint64_t ticket = 0;
    pne_options opt{};
    // owned copy of the descriptor
    std::vector<int32_t> rank, dims, bond_site, bond_leg, open_leg;
    std::vector<double> data;     // every site tensor, site after site
    std::vector<size_t> site_off;  // n_sites + 1 offsets into data
    std::vector<const double *> ptrs;
    pne_network_desc desc{};
    size_t est_bytes = 0;
    int64_t n_open_values = 0;
    Clock::time_point t_submit, t_done;
    // result
    bool done = false;
    pne_result res{};
    std::vector<double> open;
};

bool same_options(const pne_options &a, const pne_options &b) {
    return a.max_excited == b.max_excited && a.precision == b.precision && a.bp_tol == b.bp_tol &&
           a.bp_max_iter == b.bp_max_iter && a.bp_check_every == b.bp_check_every && a.flags == b.flags;
}

// Device bytes a request holds while admitted: its FP64 tensors, two FP64
// message buffers, slices in the term precision, site tables, and a bound on
// the cluster weights (one FP64 value per cluster; clusters per bond grow
// with K, bounded here by 64 per bond).
size_t estimate_bytes(const Request &r) {
    const size_t entries = r.data.size();
    size_t slots = 0;
    for (int32_t x : r.rank) slots += (size_t)x;
    const size_t esz = r.opt.precision == PNE_FP64 ? 8 : (r.opt.precision == PNE_FP32 ? 4 : 2);
    const size_t msg = 2 * 8 * 4 * slots;  // dims <= 16; generous average
    return entries * (8 + esz) + msg + 256 * r.rank.size() + 64 * 8 * (size_t)r.desc.n_bonds + 4096;
}

// A launched batch: its requests, networks and device tensors.
struct InFlight {
    pne_batch *batch = nullptr;
    void *tensors = nullptr;  // device copy of the batch's site tensors (networks borrow it)
    std::vector<pne_network *> nets;
    std::vector<Request *> reqs;
    size_t bytes = 0;
    Clock::time_point t_launch;
};

}  // namespace

struct pne_server {
    pne_ctx *ctx = nullptr;
    pne_server_options so{};
    hipStream_t streams[2] = {nullptr, nullptr};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;        // no more submissions: finish what is queued, then end the worker
    bool stop_done = false;   // the worker has ended: end the completion thread
    size_t in_use = 0;
    std::thread worker;       // admission and preparation
    std::thread launcher;     // launches prepared batches in order
    std::thread completer;    // waits for launched batches and hands out their results
    // A batch with networks swept launch by launch waits on the device
    // between its sweep chunks inside pne_batch_launch; launching on a thread
    // of its own lets the worker prepare the next batch meanwhile.
    std::condition_variable cv_launch;  // wakes the launcher
    std::deque<InFlight> to_launch;     // prepared, oldest first (the worker appends, the launcher pops)
    int launching = 0;                  // batches prepared and not yet in flight
    bool stop_launch = false;           // the worker has ended: end the launcher
    std::condition_variable cv_done;   // wakes the completion thread
    std::deque<InFlight> inflight;     // launched, oldest first (the worker appends, the completer pops)
    std::vector<InFlight> graveyard;   // finished; freed while nothing is in flight (frees synchronise)
    int64_t finished_batches = 0;
    Clock::time_point busy_since;
    // statistics
    Clock::time_point t0;
    bool any_submit = false;
    Clock::time_point t_first_submit, t_last_done;
    std::vector<double> latencies;  // seconds, completed requests
    int64_t submitted = 0, completed = 0, failed = 0, batches = 0;
    double busy_s = 0.0;
    double prep_s = 0.0;  // time creating networks and batches (worker) and launching (launcher)
    void *staging = nullptr;  // pinned upload staging of the worker
    size_t staging_bytes = 0;
    // tensor uploads run on their own stream (never behind a batch's
    // kernels); a batch stream waits on up_done, and the staging buffer is
    // rewritten only after the previous upload has completed
    hipStream_t up_stream = nullptr;
    hipEvent_t up_done = nullptr;
    bool up_pending = false;
    std::deque<uint64_t> done_q;  // finished tickets (completion_queue option)
    double wait_s = 0.0;  // worker time blocked on a batch's completion
    double upload_s = 0.0, networks_s = 0.0, batch_s = 0.0, launch_s = 0.0;  // prep_s split
    std::string err;
};

namespace {

void finish_request(pne_server *sv, Request *r, const pne_result &res, Clock::time_point t) {
    r->res = res;
    r->res.open_values = nullptr;
    r->res.open_capacity = 0;
    r->done = true;
    r->t_done = t;
    sv->latencies.push_back(seconds_since(r->t_submit, t));
    sv->t_last_done = t;
    if (res.status < 0) ++sv->failed;
    ++sv->completed;
    if (sv->so.completion_queue) sv->done_q.push_back(r->ticket);
    r->data.clear();
    r->data.shrink_to_fit();
}

void fail_request(pne_server *sv, Request *r, pne_status st) {
    pne_result res{};
    res.status = st;
    finish_request(sv, r, res, Clock::now());
}

// Copy every request's tensors to its offset in the staging buffer; a large
// batch is split into byte-balanced runs of requests copied by several
// threads (one thread's memcpy is far below the host's memory bandwidth).
void stage_tensors(char *staging, const std::vector<size_t> &toff, const std::vector<Request *> &take) {
    const size_t total = toff.back();
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({8, hw / 2 + 1, total / (4u << 20) + 1, take.size()});
    auto copy_range = [&](size_t a, size_t b) {
        for (size_t i = a; i < b; ++i)
            std::memcpy(staging + toff[i], take[i]->data.data(), take[i]->data.size() * sizeof(double));
    };
    if (nt <= 1) {
        copy_range(0, take.size());
        return;
    }
    std::vector<std::thread> th;
    size_t a = 0;
    for (size_t t = 0; t < nt && a < take.size(); ++t) {
        const size_t goal = total * (t + 1) / nt;
        size_t b = a + 1;
        while (b < take.size() && toff[b] < goal) ++b;
        if (t + 1 == nt) b = take.size();
        if (t + 1 < nt && b < take.size())
            th.emplace_back(copy_range, a, b);
        else
            copy_range(a, b);  // the last run on this thread
        a = b;
    }
    for (auto &x : th) x.join();
}

void release(pne_server *sv, InFlight &f) {
    if (f.batch) pne_batch_destroy(f.batch);
    for (pne_network *n : f.nets) pne_network_destroy(n);
    if (f.tensors) (void)hipFree(f.tensors);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->in_use -= std::min(sv->in_use, f.bytes);
}

// Upload the requests' tensors and create their networks and one batch on
// stream s.  Requests that fail are finished here; false when no batch was
// made (f then holds whatever must be released).
bool prepare_batch(pne_server *sv, const std::vector<Request *> &take, hipStream_t s, InFlight &f) {
    const Clock::time_point tp0 = Clock::now();
    for (Request *r : take) f.bytes += r->est_bytes;
    // every request's tensors in one device allocation, uploaded by one copy
    // from the server's pinned staging buffer on the upload stream; the batch
    // stream waits for it
    std::vector<size_t> toff(take.size() + 1, 0);
    for (size_t i = 0; i < take.size(); ++i) {
        const size_t b = take[i]->data.size() * sizeof(double);
        toff[i + 1] = toff[i] + ((b + 255) & ~(size_t)255);
    }
    pne_status ust = PNE_OK;
    if (sv->up_pending) {  // the previous upload still reads the staging buffer
        if (hipEventSynchronize(sv->up_done) != hipSuccess) ust = PNE_ERR_DEVICE;
        sv->up_pending = false;
    }
    if (ust == PNE_OK && hipMalloc(&f.tensors, std::max<size_t>(toff.back(), 256)) != hipSuccess) {
        f.tensors = nullptr;
        ust = PNE_ERR_OUT_OF_MEMORY;
    }
    if (ust == PNE_OK && sv->staging_bytes < toff.back()) {
        if (sv->staging) (void)hipHostFree(sv->staging);
        sv->staging = nullptr;
        sv->staging_bytes = 0;
        const size_t want = std::max(toff.back() + toff.back() / 2, (size_t)1 << 22);
        if (hipHostMalloc(&sv->staging, want, hipHostMallocDefault) == hipSuccess)
            sv->staging_bytes = want;
        else
            ust = PNE_ERR_OUT_OF_MEMORY;
    }
    if (ust == PNE_OK) {
        stage_tensors((char *)sv->staging, toff, take);
        if (hipMemcpyAsync(f.tensors, sv->staging, toff.back(), hipMemcpyHostToDevice, sv->up_stream) !=
                hipSuccess ||
            hipEventRecord(sv->up_done, sv->up_stream) != hipSuccess ||
            hipStreamWaitEvent(s, sv->up_done, 0) != hipSuccess)
            ust = PNE_ERR_DEVICE;
        else
            sv->up_pending = true;
    }
    const Clock::time_point tp1 = Clock::now();
    std::vector<Request *> ok;
    std::vector<const double *> dptr;
    for (size_t i = 0; i < take.size(); ++i) {
        Request *r = take[i];
        pne_network *n = nullptr;
        pne_status st = ust;
        if (st == PNE_OK) {
            const size_t ns = r->rank.size();
            dptr.resize(ns);
            const double *d = (const double *)((const char *)f.tensors + toff[i]);
            for (size_t k = 0; k < ns; ++k) dptr[k] = d + r->site_off[k];
            pne_network_desc dd = r->desc;
            dd.site_data = dptr.data();
            st = pne::network_create_on(sv->ctx, &dd, 1, s, &n);
        }
        if (st != PNE_OK) {
            std::lock_guard<std::mutex> lk(sv->mu);
            fail_request(sv, r, st);
            continue;
        }
        f.nets.push_back(n);
        ok.push_back(r);
    }
    f.reqs = ok;
    const Clock::time_point tp2 = Clock::now();
    if (f.nets.empty()) return false;
    pne_status st = pne::batch_create_on(sv->ctx, f.nets.data(), (int32_t)f.nets.size(), &ok[0]->opt, s, &f.batch);
    const Clock::time_point tp3 = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (st != PNE_OK) {
        for (Request *r : ok) fail_request(sv, r, st);
        return false;
    }
    sv->prep_s += seconds_since(tp0, tp3);
    sv->upload_s += seconds_since(tp0, tp1);
    sv->networks_s += seconds_since(tp1, tp2);
    sv->batch_s += seconds_since(tp2, tp3);
    return true;
}

// Launch: takes prepared batches in order and launches them; a launched
// batch goes to the completion thread, a failed one to the graveyard.  At
// most pipeline_depth (<= 2) batches are being launched or in flight, on the
// server's two streams.
void launcher_main(pne_server *sv) {
    for (;;) {
        InFlight f;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_launch.wait(lk, [&] { return sv->stop_launch || !sv->to_launch.empty(); });
            if (sv->to_launch.empty()) break;  // stop_launch
            f = std::move(sv->to_launch.front());
            sv->to_launch.pop_front();
        }
        const Clock::time_point tl0 = Clock::now();
        const pne_status st = pne_batch_launch(f.batch);
        const Clock::time_point tl1 = Clock::now();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->prep_s += seconds_since(tl0, tl1);
            sv->launch_s += seconds_since(tl0, tl1);
            --sv->launching;
            if (st != PNE_OK) {
                for (Request *r : f.reqs) fail_request(sv, r, st);
                sv->graveyard.push_back(std::move(f));
            } else {
                f.t_launch = tl1;
                if (sv->inflight.empty()) sv->busy_since = f.t_launch;
                sv->inflight.push_back(std::move(f));
                ++sv->batches;
            }
        }
        sv->cv_done.notify_all();
        sv->cv.notify_all();
    }
}

// Admission and preparation: takes pending requests in arrival order while
// their estimated bytes fit the budget and fewer than pipeline_depth
// batches are being launched or in flight, prepares them and hands them to
// the launcher, and frees finished batches whenever nothing is being
// launched or in flight.
constexpr int kGraveyardMax = 8;

void worker_main(pne_server *sv) {
    int launch_count = 0;
    const int depth = sv->so.pipeline_depth;
    for (;;) {
        std::vector<Request *> take;
        std::vector<InFlight> dead;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            int64_t seen = sv->finished_batches;
            bool blocked = false;  // the oldest pending request waits for memory
            for (;;) {
                // finished batches are freed while nothing is in flight (a free
                // synchronises the device), or once kGraveyardMax pile up
                auto idle = [&] { return sv->inflight.empty() && sv->launching == 0; };
                auto release_now = [&] {
                    return !sv->graveyard.empty() && (idle() || (int)sv->graveyard.size() >= kGraveyardMax);
                };
                const auto active = [&] { return (int)sv->inflight.size() + sv->launching; };
                sv->cv.wait(lk, [&] {
                    return (!blocked && active() < depth && !sv->pending.empty()) || release_now() ||
                           (sv->stop && sv->pending.empty() && idle()) || sv->finished_batches != seen;
                });
                if (sv->finished_batches != seen) blocked = false;
                seen = sv->finished_batches;
                if (release_now()) {
                    dead.swap(sv->graveyard);
                    break;
                }
                if (sv->stop && sv->pending.empty() && idle()) break;
                if (active() >= depth || sv->pending.empty()) continue;
                const pne_options head = sv->pending.front()->opt;
                size_t bytes = 0;
                for (auto it = sv->pending.begin(); it != sv->pending.end() && (int)take.size() < sv->so.max_batch;) {
                    Request *r = *it;
                    const bool fits =
                        sv->so.mem_budget == 0 || sv->in_use + bytes + r->est_bytes <= sv->so.mem_budget;
                    if (same_options(r->opt, head) && (fits || (idle() && take.empty() && sv->in_use == 0))) {
                        take.push_back(r);
                        bytes += r->est_bytes;
                        it = sv->pending.erase(it);
                    } else if (!fits) {
                        break;  // arrival order: later requests wait behind one that does not fit
                    } else {
                        ++it;
                    }
                }
                if (!take.empty()) {
                    sv->in_use += bytes;
                    break;
                }
                blocked = true;  // nothing fits until a batch finishes and is freed
            }
            if (dead.empty() && take.empty()) break;  // stopped and drained
        }
        if (!dead.empty()) {
            for (InFlight &f : dead) release(sv, f);
            continue;
        }
        InFlight f;
        hipStream_t s = sv->streams[launch_count % 2];
        if (!prepare_batch(sv, take, s, f)) {
            release(sv, f);
            continue;
        }
        ++launch_count;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->to_launch.push_back(std::move(f));
            ++sv->launching;
        }
        sv->cv_launch.notify_all();
    }
    if (sv->up_stream) (void)hipStreamSynchronize(sv->up_stream);
    if (sv->staging) (void)hipHostFree(sv->staging);
    sv->staging = nullptr;
}

// Completion: waits for the oldest launched batch, hands its results to its
// requests as soon as the device is done (while the worker prepares the next
// batch), and moves the batch to the graveyard.
void completer_main(pne_server *sv) {
    for (;;) {
        InFlight *fp = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_done.wait(lk, [&] { return sv->stop_done || !sv->inflight.empty(); });
            if (sv->inflight.empty()) break;  // stop_done
            fp = &sv->inflight.front();       // stays put: the worker only appends
        }
        InFlight &f = *fp;
        const size_t n = f.reqs.size();
        std::vector<pne_result> res(n);
        for (size_t i = 0; i < n; ++i) {
            std::memset(&res[i], 0, sizeof res[i]);
            f.reqs[i]->open.assign((size_t)std::max<int64_t>(f.reqs[i]->n_open_values, 1), 0.0);
            res[i].open_values = f.reqs[i]->open.data();
            res[i].open_capacity = f.reqs[i]->n_open_values;
        }
        const Clock::time_point tw0 = Clock::now();
        pne_status st = pne_batch_wait(f.batch, res.data());
        const Clock::time_point t = Clock::now();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->wait_s += seconds_since(tw0, t);
            for (size_t i = 0; i < n; ++i) {
                if (st < 0 && res[i].status >= 0 && st != PNE_ERR_SINGULAR && st != PNE_ERR_INVALID_ARG)
                    res[i].status = st;  // device error: no result for anyone
                finish_request(sv, f.reqs[i], res[i], t);
            }
            sv->graveyard.push_back(std::move(sv->inflight.front()));
            sv->inflight.pop_front();
            if (sv->inflight.empty()) sv->busy_s += seconds_since(sv->busy_since, t);
            ++sv->finished_batches;
        }
        sv->cv.notify_all();
    }
}

}  // namespace

extern "C" {

pne_status pne_server_options_default(pne_server_options *o) {
    if (!o) return PNE_ERR_INVALID_ARG;
    std::memset(o, 0, sizeof *o);
    o->mem_budget = 0;
    o->max_batch = 1024;
    o->pipeline_depth = 2;
    return PNE_OK;
}

pne_status pne_server_create(pne_ctx *ctx, const pne_server_options *opt, pne_server **out) {
    if (!ctx || !out) return PNE_ERR_INVALID_ARG;
    *out = nullptr;
    auto sv = std::make_unique<pne_server>();
    sv->ctx = ctx;
    pne_server_options_default(&sv->so);
    if (opt) sv->so = *opt;
    if (sv->so.max_batch <= 0) sv->so.max_batch = 1024;
    if (sv->so.pipeline_depth < 1) sv->so.pipeline_depth = 1;
    if (sv->so.pipeline_depth > 2) sv->so.pipeline_depth = 2;
    for (hipStream_t *s : {&sv->streams[0], &sv->streams[1], &sv->up_stream})
        if (hipStreamCreateWithFlags(s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : {sv->streams[0], sv->streams[1], sv->up_stream})
                if (t) (void)hipStreamDestroy(t);
            return PNE_ERR_DEVICE;
        }
    if (hipEventCreateWithFlags(&sv->up_done, hipEventDisableTiming) != hipSuccess) {
        for (hipStream_t t : {sv->streams[0], sv->streams[1], sv->up_stream}) (void)hipStreamDestroy(t);
        return PNE_ERR_DEVICE;
    }
    sv->t0 = Clock::now();
    pne_server *p = sv.release();
    int dev = 0;
    (void)hipGetDevice(&dev);
    p->worker = std::thread([p, dev] {
        (void)hipSetDevice(dev);
        worker_main(p);
    });
    p->launcher = std::thread([p, dev] {
        (void)hipSetDevice(dev);
        launcher_main(p);
    });
    p->completer = std::thread([p, dev] {
        (void)hipSetDevice(dev);
        completer_main(p);
    });
    *out = p;
    return PNE_OK;
}

pne_status pne_server_destroy(pne_server *sv) {
    if (!sv) return PNE_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();  // every request finished, every batch freed
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop_launch = true;
    }
    sv->cv_launch.notify_all();
    if (sv->launcher.joinable()) sv->launcher.join();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop_done = true;
    }
    sv->cv_done.notify_all();
    if (sv->completer.joinable()) sv->completer.join();
    for (hipStream_t t : {sv->streams[0], sv->streams[1], sv->up_stream})
        if (t) (void)hipStreamDestroy(t);
    if (sv->up_done) (void)hipEventDestroy(sv->up_done);
    delete sv;
    return PNE_OK;
}

pne_status pne_submit(pne_server *sv, const pne_network_desc *d, const pne_options *opt, uint64_t *ticket) {
    if (!sv || !d || !opt || !ticket) return PNE_ERR_INVALID_ARG;
    if (d->n_sites <= 0 || d->n_bonds < 0 || d->n_open < 0 || !d->site_rank || !d->leg_dim || !d->site_data ||
        (d->n_bonds > 0 && (!d->bond_site || !d->bond_leg)) || (d->n_open > 0 && !d->open_leg))
        return PNE_ERR_INVALID_ARG;
    auto r = std::make_unique<Request>();
    r->opt = *opt;
    r->rank.assign(d->site_rank, d->site_rank + d->n_sites);
    size_t n_slots = 0;
    for (int32_t x : r->rank) {
        if (x < 0 || x > 8) return PNE_ERR_INVALID_ARG;
        n_slots += (size_t)x;
    }
    r->dims.assign(d->leg_dim, d->leg_dim + n_slots);
    r->bond_site.assign(d->bond_site, d->bond_site + 2 * (size_t)d->n_bonds);
    r->bond_leg.assign(d->bond_leg, d->bond_leg + 2 * (size_t)d->n_bonds);
    if (d->n_open > 0) r->open_leg.assign(d->open_leg, d->open_leg + 2 * (size_t)d->n_open);
    r->site_off.assign(d->n_sites + 1, 0);
    size_t slot = 0;
    int64_t n_open_values = 1;
    for (int s = 0; s < d->n_sites; ++s) {
        size_t size = 1;
        for (int l = 0; l < r->rank[s]; ++l) {
            if (r->dims[slot + l] <= 0) return PNE_ERR_INVALID_ARG;
            size *= (size_t)r->dims[slot + l];
        }
        if (!d->site_data[s]) return PNE_ERR_INVALID_ARG;
        r->site_off[s + 1] = r->site_off[s] + size;
        slot += r->rank[s];
    }
    r->data.resize(r->site_off.back());
    r->ptrs.resize(d->n_sites);
    for (int s = 0; s < d->n_sites; ++s) {
        const size_t size = r->site_off[s + 1] - r->site_off[s];
        double *dst = r->data.data() + r->site_off[s];
        std::memcpy(dst, d->site_data[s], size * sizeof(double));
        for (size_t i = 0; i < size; ++i)
            if (!std::isfinite(dst[i])) return PNE_ERR_INVALID_ARG;
        r->ptrs[s] = dst;
    }
    for (int k = 0; k < d->n_open; ++k) {
        const int s = r->open_leg[2 * k], l = r->open_leg[2 * k + 1];
        if (s < 0 || s >= d->n_sites || l < 0 || l >= r->rank[s]) return PNE_ERR_INVALID_ARG;
        size_t base = 0;
        for (int t = 0; t < s; ++t) base += r->rank[t];
        n_open_values *= r->dims[base + l];
    }
    r->n_open_values = d->n_open > 0 ? n_open_values : 0;
    r->desc = *d;
    r->desc.site_rank = r->rank.data();
    r->desc.leg_dim = r->dims.data();
    r->desc.bond_site = r->bond_site.empty() ? nullptr : r->bond_site.data();
    r->desc.bond_leg = r->bond_leg.empty() ? nullptr : r->bond_leg.data();
    r->desc.open_leg = r->open_leg.empty() ? nullptr : r->open_leg.data();
    r->desc.site_data = r->ptrs.data();
    r->est_bytes = estimate_bytes(*r);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->so.mem_budget && r->est_bytes > sv->so.mem_budget) return PNE_ERR_OUT_OF_MEMORY;
        r->ticket = sv->next_ticket++;
        *ticket = r->ticket;
        if (!sv->any_submit) {
            sv->any_submit = true;
            sv->t_first_submit = r->t_submit;
        }
        ++sv->submitted;
        sv->pending.push_back(r.get());
        sv->all.emplace(r->ticket, std::move(r));
    }
    sv->cv.notify_all();
    return PNE_OK;
}

pne_status pne_poll(pne_server *sv, uint64_t ticket, pne_result *res) {
    if (!sv || !res) return PNE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return PNE_ERR_INVALID_ARG;
    Request *r = it->second.get();
    if (!r->done) return PNE_ERR_NOT_READY;
    double *ov = res->open_values;
    const int64_t cap = res->open_capacity;
    *res = r->res;
    res->open_values = ov;
    res->open_capacity = cap;
    res->n_open_values = 0;
    if (r->res.status >= 0 && r->n_open_values > 0) {
        if (!ov || cap < r->n_open_values) return PNE_ERR_INVALID_ARG;  // result kept; poll again
        std::memcpy(ov, r->open.data(), sizeof(double) * (size_t)r->n_open_values);
        res->n_open_values = (int32_t)r->n_open_values;
    }
    const pne_status st = (pne_status)r->res.status;
    sv->all.erase(it);
    return st;
}

pne_status pne_cancel(pne_server *sv, uint64_t ticket) {
    if (!sv) return PNE_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->all.find(ticket);
        if (it == sv->all.end() || it->second->done) return PNE_ERR_INVALID_ARG;
        Request *r = it->second.get();
        auto q = std::find(sv->pending.begin(), sv->pending.end(), r);
        if (q == sv->pending.end()) return PNE_ERR_NOT_READY;  // admitted: it runs to completion
        sv->pending.erase(q);
        r->res = pne_result{};
        r->res.status = PNE_ERR_CANCELLED;
        r->done = true;
        r->t_done = Clock::now();
        ++sv->failed;
        ++sv->completed;
        if (sv->so.completion_queue) sv->done_q.push_back(r->ticket);
        r->data.clear();
        r->data.shrink_to_fit();
    }
    sv->cv.notify_all();  // the queue's head may have changed (memory admission)
    return PNE_OK;
}

pne_status pne_server_get_stats(pne_server *sv, pne_server_stats *out) {
    if (!sv || !out) return PNE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->failed = sv->failed;
    out->batches = sv->batches;
    out->pending = (int64_t)sv->pending.size();
    out->device_bytes_admitted = (int64_t)sv->in_use;
    out->busy_s = sv->busy_s;
    out->prep_s = sv->prep_s;
    out->wait_s = sv->wait_s;
    out->upload_s = sv->upload_s;
    out->networks_s = sv->networks_s;
    out->batch_s = sv->batch_s;
    out->launch_s = sv->launch_s;
    if (!sv->latencies.empty()) {
        std::vector<double> l = sv->latencies;
        std::sort(l.begin(), l.end());
        auto q = [&](double p) {
            const double x = p * (double)(l.size() - 1);
            const size_t i = (size_t)x;
            const double f = x - (double)i;
            return i + 1 < l.size() ? l[i] * (1.0 - f) + l[i + 1] * f : l[i];
        };
        double s = 0.0;
        for (double v : l) s += v;
        out->latency_p50_ms = 1e3 * q(0.50);
        out->latency_p99_ms = 1e3 * q(0.99);
        out->latency_mean_ms = 1e3 * s / (double)l.size();
        out->latency_max_ms = 1e3 * l.back();
        const double span = seconds_since(sv->t_first_submit, sv->t_last_done);
        out->networks_per_s = span > 0 ? (double)sv->completed / span : 0.0;
    }
    return PNE_OK;
}

pne_status pne_server_completed(pne_server *sv, uint64_t *tickets, int32_t capacity, int32_t *n) {
    if (!sv || !tickets || !n || capacity < 0 || !sv->so.completion_queue) return PNE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    int32_t k = 0;
    while (k < capacity && !sv->done_q.empty()) {
        tickets[k++] = sv->done_q.front();
        sv->done_q.pop_front();
    }
    *n = k;
    return PNE_OK;
}

}  // extern "C"
