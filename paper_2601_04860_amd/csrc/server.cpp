// Continuous-batching server for click-driven view updates (the per-update
// re-fusion of the paper's interaction loop, served for many sessions).
//
// Written against the public C ABI only.  One scheduler thread owns every HIP
// call on the server's sessions:
//   * completion: in-flight batches (one per stream slot) are polled through
//     their completion events; each request's latency is the time from its
//     arrival stamp to the moment its batch's completion is observed;
//   * admission: session opens wait in FIFO order until the session's HBM
//     footprint fits the context's budget; closing sessions free their share
//     once their requests are done;
//   * dispatch: whenever a stream slot is free, the queued requests of admitted
//     sessions without work in flight are gathered (FIFO, one request per
//     session) into one batched launch on that slot's stream, so requests that
//     arrive while others run join the next batch and batches on different
//     slots overlap on the device.
// A session's requests are applied in submission order and each request's
// outputs are bit-identical to applying it alone (see divas_batch_run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <new>
#include <thread>
#include <vector>

#include "../../include/divas.h"

namespace {

using clk = std::chrono::steady_clock;

struct Req {
    uint64_t ticket = 0;
    int sid = 0;
    int op = 0;
    int32_t slot = 0;
    std::vector<divas_camera> cams;
    std::vector<divas_view_maps> maps;
    divas_result out{};
    double arrival = 0, launched = 0, done = 0;
    int state = 0;  // 0 queued, 1 in flight, 2 done, 3 failed
    divas_status status = DIVAS_OK;
};

struct SessRec {
    int sid = 0;
    divas_session s = nullptr;
    bool admitted = false, closing = false, closed = false, busy = false, failed = false;
    divas_grid grid{};
    divas_occupancy occ{};
    divas_params params{};
    int64_t max_points = 0;
    int32_t max_views = 0;
    int64_t max_pix = 0;
    size_t footprint = 0;
    int queued = 0;  // requests not yet done
    double open_request = 0, admitted_at = 0;
};

struct Slot {
    divas_batch b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> reqs;
    std::vector<int> sids;
};

}  // namespace

struct divas_server_s {
    divas_ctx ctx = nullptr;
    int device = 0;
    int32_t max_batch = 64, max_new_views = 64;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    clk::time_point t0;
    std::map<uint64_t, Req> reqs;
    std::deque<uint64_t> fifo;
    std::map<int, SessRec> sess;
    std::deque<int> admit_q;
    std::vector<Slot> slots;
    hipStream_t admin = nullptr;
    uint64_t next_ticket = 1;
    int next_sid = 1;
    // statistics
    int64_t batches = 0, batched_requests = 0, admission_waits = 0, max_queue = 0, failures = 0;
    std::vector<double> lat_ms;  // update requests
    std::string last_error;

    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
};


namespace {

void set_err(divas_server_s* S, const char* m) { S->last_error = m; }

// Called with the lock held.
void complete_slot(divas_server_s* S, Slot& sl, bool ok) {
    double t = S->now();
    for (uint64_t k : sl.reqs) {
        auto it = S->reqs.find(k);
        if (it == S->reqs.end()) continue;
        Req& r = it->second;
        r.done = t;
        r.state = ok ? 2 : 3;
        if (!ok) ++S->failures;
        if (ok && r.op == DIVAS_BATCH_UPDATE) S->lat_ms.push_back((r.done - r.arrival) * 1e3);
        auto si = S->sess.find(r.sid);
        if (si != S->sess.end()) si->second.queued -= 1;
    }
    for (int sid : sl.sids) {
        auto si = S->sess.find(sid);
        if (si != S->sess.end()) si->second.busy = false;
    }
    sl.reqs.clear();
    sl.sids.clear();
    sl.busy = false;
}

bool poll_completions(divas_server_s* S) {
    bool any = false;
    for (auto& sl : S->slots) {
        if (!sl.busy) continue;
        hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) continue;
        complete_slot(S, sl, e == hipSuccess);
        any = true;
    }
    return any;
}

// Admit waiting sessions (FIFO) whose footprint fits; destroy drained closing sessions.
bool admission(divas_server_s* S) {
    bool any = false;
    for (auto it = S->sess.begin(); it != S->sess.end();) {
        SessRec& r = it->second;
        if (r.closing && r.admitted && !r.busy && r.queued == 0) {
            if (r.s) (void)divas_session_destroy(r.s);
            r.s = nullptr;
            r.closed = true;
            it = S->sess.erase(it);
            any = true;
            continue;
        }
        ++it;
    }
    while (!S->admit_q.empty()) {
        int sid = S->admit_q.front();
        auto it = S->sess.find(sid);
        if (it == S->sess.end()) {
            S->admit_q.pop_front();
            continue;
        }
        SessRec& r = it->second;
        size_t used = 0, budget = 0;
        (void)divas_ctx_usage(S->ctx, &used, &budget);
        if (budget && used + r.footprint > budget) {
            ++S->admission_waits;
            break;  // FIFO: the head waits for memory
        }
        divas_status st = divas_session_create(S->ctx, &r.grid, &r.occ, &r.params, r.max_points, r.max_views,
                                               r.max_pix, S->admin, &r.s);
        if (st == DIVAS_ERR_ADMISSION) {
            ++S->admission_waits;
            break;
        }
        S->admit_q.pop_front();
        if (st != DIVAS_OK) {
            r.failed = true;
            r.s = nullptr;
        } else {
            (void)hipStreamSynchronize(S->admin);
            r.admitted = true;
            r.admitted_at = S->now();
        }
        any = true;
    }
    return any;
}

// On stop, sessions still waiting for admission are given up: their queued
// requests fail (the sessions admitted so far may hold the memory until the
// end, so waiting could last for ever).  Called with the lock held.
bool give_up_waiting(divas_server_s* S) {
    if (!S->stop) return false;
    bool any = false;
    for (auto it = S->fifo.begin(); it != S->fifo.end();) {
        Req& r = S->reqs[*it];
        auto si = S->sess.find(r.sid);
        if (si != S->sess.end() && si->second.admitted) {
            ++it;
            continue;
        }
        r.state = 3;
        r.status = DIVAS_ERR_ADMISSION;
        r.done = S->now();
        ++S->failures;
        if (si != S->sess.end()) si->second.queued -= 1;
        it = S->fifo.erase(it);
        any = true;
    }
    for (auto& kv : S->sess)
        if (!kv.second.admitted) kv.second.failed = true;
    S->admit_q.clear();
    return any;
}

// Gather one batch for a free slot.  Called with the lock held; returns false
// when nothing is eligible.
bool dispatch(divas_server_s* S, std::unique_lock<std::mutex>& lk) {
    Slot* free_slot = nullptr;
    for (auto& sl : S->slots)
        if (!sl.busy) {
            free_slot = &sl;
            break;
        }
    if (!free_slot || S->fifo.empty()) return false;
    std::vector<uint64_t> take;
    std::vector<int> sids;
    std::vector<int> seen;
    int views = 0;
    for (auto it = S->fifo.begin(); it != S->fifo.end() && (int)take.size() < S->max_batch;) {
        Req& r = S->reqs[*it];
        auto si = S->sess.find(r.sid);
        bool drop = si == S->sess.end() || si->second.failed;
        if (drop) {  // session gone or failed: the request fails
            r.state = 3;
            r.status = DIVAS_ERR_STATE;
            ++S->failures;
            if (si != S->sess.end()) si->second.queued -= 1;
            it = S->fifo.erase(it);
            continue;
        }
        SessRec& sr = si->second;
        bool blocked = !sr.admitted || sr.busy || std::find(seen.begin(), seen.end(), r.sid) != seen.end();
        int nv = (int)r.cams.size();
        if (blocked || views + nv > S->max_new_views) {
            // keep the session's order: later requests of a blocked session wait too
            if (std::find(seen.begin(), seen.end(), r.sid) == seen.end()) seen.push_back(r.sid);
            ++it;
            continue;
        }
        seen.push_back(r.sid);
        take.push_back(*it);
        sids.push_back(r.sid);
        views += nv;
        it = S->fifo.erase(it);
    }
    if (take.empty()) return false;
    std::vector<divas_batch_item> items;
    std::vector<uint64_t> good;
    std::vector<int> good_sids;
    items.reserve(take.size());
    double t = S->now();
    for (size_t k = 0; k < take.size(); ++k) {
        Req& r = S->reqs[take[k]];
        SessRec& sr = S->sess[r.sid];
        divas_batch_item it;
        std::memset(&it, 0, sizeof it);
        it.session = sr.s;
        it.op = r.op;
        it.n_views = (int32_t)r.cams.size();
        it.slot = r.slot;
        if (r.op == DIVAS_BATCH_UPDATE && r.slot < 0) {
            int32_t nv = 0;
            (void)divas_session_info(sr.s, nullptr, nullptr, &nv, nullptr);
            it.slot = nv;  // append
        }
        it.cams = r.cams.data();
        it.maps = r.maps.data();
        it.out = r.out;
        // an invalid request (a slot past max_views, a bad camera, ...) fails
        // alone instead of failing the requests batched with it
        divas_status vs = divas_batch_validate(free_slot->b, 1, &it);
        if (vs != DIVAS_OK) {
            set_err(S, divas_last_error());
            r.state = 3;
            r.status = vs;
            r.done = t;
            ++S->failures;
            sr.queued -= 1;
            continue;
        }
        sr.busy = true;
        r.state = 1;
        r.launched = t;
        items.push_back(it);
        good.push_back(take[k]);
        good_sids.push_back(r.sid);
    }
    take.swap(good);
    sids.swap(good_sids);
    if (take.empty()) return true;  // every request failed validation (progress all the same)
    Slot& sl = *free_slot;
    sl.busy = true;
    sl.reqs = take;
    sl.sids = sids;
    // the batch call issues HIP work; submitters may proceed meanwhile (only the
    // scheduler touches sessions and slots)
    lk.unlock();
    divas_status st = divas_batch_run(sl.b, (int32_t)items.size(), items.data(), sl.st);
    hipError_t he = hipSuccess;
    if (st == DIVAS_OK) he = hipEventRecord(sl.done, sl.st);
    lk.lock();
    S->batches += 1;
    S->batched_requests += (int64_t)take.size();
    if (st != DIVAS_OK || he != hipSuccess) {
        set_err(S, divas_last_error());
        for (uint64_t k : take) S->reqs[k].status = st != DIVAS_OK ? st : DIVAS_ERR_DEVICE;
        complete_slot(S, sl, false);
    }
    return true;
}

void scheduler(divas_server_s* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = poll_completions(S);
        progress |= admission(S);
        progress |= give_up_waiting(S);
        while (dispatch(S, lk)) progress = true;
        if (progress) S->cv.notify_all();
        bool inflight = false;
        for (auto& sl : S->slots) inflight |= sl.busy;
        if (S->stop && !inflight && S->fifo.empty()) break;
        if (inflight)
            S->cv.wait_for(lk, std::chrono::microseconds(20));
        else if (!progress)
            S->cv.wait_for(lk, std::chrono::milliseconds(2));
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    double pos = q * (double)(v.size() - 1);
    size_t i = (size_t)pos;
    double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

divas_status divas_server_create(divas_ctx ctx, const divas_server_config* cfg, divas_server* out) {
    if (!out || !ctx) return DIVAS_ERR_ARG;
    *out = nullptr;
    divas_server_config c{};
    c.n_streams = 2;
    c.max_batch = 64;
    c.max_new_views = 64;
    c.batch.use_graph = 1;
    if (cfg) c = *cfg;
    if (c.n_streams < 1 || c.n_streams > 8 || c.max_batch < 1 || c.max_new_views < 1) return DIVAS_ERR_ARG;
    divas_server_s* S = new (std::nothrow) divas_server_s;
    if (!S) return DIVAS_ERR_OOM;
    S->ctx = ctx;
    S->max_batch = c.max_batch;
    S->max_new_views = c.max_new_views;
    S->t0 = clk::now();
    int dev = 0;
    (void)hipGetDevice(&dev);
    S->device = dev;
    bool ok = hipStreamCreateWithFlags(&S->admin, hipStreamNonBlocking) == hipSuccess;
    S->slots.resize(c.n_streams);
    for (auto& sl : S->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
             divas_batch_create(ctx, c.max_batch, c.max_new_views, &c.batch, &sl.b) == DIVAS_OK;
    }
    if (!ok) {
        for (auto& sl : S->slots) {
            if (sl.b) (void)divas_batch_destroy(sl.b);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.st) (void)hipStreamDestroy(sl.st);
        }
        if (S->admin) (void)hipStreamDestroy(S->admin);
        delete S;
        return DIVAS_ERR_DEVICE;
    }
    S->th = std::thread(scheduler, S);
    *out = S;
    return DIVAS_OK;
}

double divas_server_now(divas_server S) { return S ? S->now() : 0.0; }

divas_status divas_server_open_session(divas_server S, const divas_grid* grid, const divas_occupancy* occ,
                                       const divas_params* params, int64_t max_points, int32_t max_views,
                                       int64_t max_view_pixels, int32_t* session_id) {
    if (!S || !grid || !occ || !params || !session_id) return DIVAS_ERR_ARG;
    size_t fp = divas_session_footprint(grid, max_points > 0 ? max_points : occ->n, max_views, max_view_pixels,
                                        params->retain_state || params->differentiable);
    if (fp == 0) return DIVAS_ERR_ARG;
    if (params->thin) {  // the thin path's point counts per active voxel
        const int64_t nvox = (int64_t)grid->dim * grid->dim * grid->dim;
        const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(max_points > 0 ? max_points : occ->n, nvox));
        fp += ((size_t)cap * 4 + 255) / 256 * 256;
    }
    size_t used = 0, budget = 0;
    (void)divas_ctx_usage(S->ctx, &used, &budget);
    // a session larger than the whole budget could never be admitted and would
    // hold the head of the admission queue for ever
    if (budget && fp > budget) return DIVAS_ERR_ADMISSION;
    std::lock_guard<std::mutex> g(S->mu);
    SessRec r;
    r.sid = S->next_sid++;
    r.grid = *grid;
    r.occ = *occ;
    r.params = *params;
    r.max_points = max_points;
    r.max_views = max_views;
    r.max_pix = max_view_pixels;
    r.footprint = fp;
    r.open_request = S->now();
    S->sess[r.sid] = r;
    S->admit_q.push_back(r.sid);
    *session_id = r.sid;
    S->cv.notify_all();
    return DIVAS_OK;
}

divas_status divas_server_session(divas_server S, int32_t sid, divas_session* out, int32_t* admitted) {
    if (!S) return DIVAS_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->sess.find(sid);
    if (it == S->sess.end()) return DIVAS_ERR_STATE;
    if (out) *out = it->second.s;
    if (admitted) *admitted = it->second.admitted ? 1 : (it->second.failed ? -1 : 0);
    return DIVAS_OK;
}

divas_status divas_server_close_session(divas_server S, int32_t sid) {
    if (!S) return DIVAS_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->sess.find(sid);
    if (it == S->sess.end()) return DIVAS_ERR_STATE;
    it->second.closing = true;
    S->cv.notify_all();
    return DIVAS_OK;
}

divas_status divas_server_submit(divas_server S, int32_t sid, int32_t op, int32_t n_views, int32_t slot,
                                 const divas_camera* cams, const divas_view_maps* maps, const divas_result* out,
                                 double arrival, uint64_t* ticket) {
    if (!S || !cams || !maps || !out || !ticket || n_views < 1) return DIVAS_ERR_ARG;
    if (op != DIVAS_BATCH_FUSE && op != DIVAS_BATCH_UPDATE) return DIVAS_ERR_ARG;
    if (op == DIVAS_BATCH_UPDATE && n_views != 1) return DIVAS_ERR_ARG;
    if (n_views > S->max_new_views) return DIVAS_ERR_CAPACITY;
    std::lock_guard<std::mutex> g(S->mu);
    auto si = S->sess.find(sid);
    if (si == S->sess.end() || si->second.closing) return DIVAS_ERR_STATE;
    Req r;
    r.ticket = S->next_ticket++;
    r.sid = sid;
    r.op = op;
    r.slot = slot;
    r.cams.assign(cams, cams + n_views);
    r.maps.assign(maps, maps + n_views);
    r.out = *out;
    r.arrival = arrival >= 0 ? arrival : S->now();
    si->second.queued += 1;
    S->reqs[r.ticket] = std::move(r);
    S->fifo.push_back(r.ticket);
    S->max_queue = std::max<int64_t>(S->max_queue, (int64_t)S->fifo.size());
    *ticket = S->next_ticket - 1;
    S->cv.notify_all();
    return DIVAS_OK;
}

divas_status divas_server_wait(divas_server S, uint64_t ticket, double timeout_s, int32_t* done, double* latency_ms) {
    if (!S) return DIVAS_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto pred = [&]() {
        auto it = S->reqs.find(ticket);
        return it == S->reqs.end() || it->second.state >= 2;
    };
    if (timeout_s > 0)
        S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return DIVAS_ERR_ARG;
    const Req& r = it->second;
    if (done) *done = r.state >= 2 ? 1 : 0;
    if (latency_ms) *latency_ms = r.state >= 2 ? (r.done - r.arrival) * 1e3 : -1.0;
    return r.state == 3 ? (r.status != DIVAS_OK ? r.status : DIVAS_ERR_DEVICE) : DIVAS_OK;
}

divas_status divas_server_drain(divas_server S, double timeout_s) {
    if (!S) return DIVAS_ERR_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    bool ok = S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&]() {
        bool inflight = false;
        for (auto& sl : S->slots) inflight |= sl.busy;
        return S->fifo.empty() && !inflight;
    });
    return ok ? DIVAS_OK : DIVAS_ERR_STATE;
}

divas_status divas_server_stats(divas_server S, divas_server_statistics* st) {
    if (!S || !st) return DIVAS_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    std::memset(st, 0, sizeof *st);
    st->completed_updates = (int64_t)S->lat_ms.size();
    st->batches = S->batches;
    st->batched_requests = S->batched_requests;
    st->admission_waits = S->admission_waits;
    st->max_queue = S->max_queue;
    st->failures = S->failures;
    st->p50_ms = percentile(S->lat_ms, 0.50);
    st->p99_ms = percentile(S->lat_ms, 0.99);
    st->max_ms = S->lat_ms.empty() ? 0.0 : *std::max_element(S->lat_ms.begin(), S->lat_ms.end());
    double sum = 0;
    for (double x : S->lat_ms) sum += x;
    st->mean_ms = S->lat_ms.empty() ? 0.0 : sum / (double)S->lat_ms.size();
    int64_t open = 0, waiting = 0;
    for (auto& kv : S->sess) {
        open += kv.second.admitted ? 1 : 0;
        waiting += kv.second.admitted ? 0 : 1;
    }
    st->sessions_open = open;
    st->sessions_waiting = waiting;
    return DIVAS_OK;
}

divas_status divas_server_latencies(divas_server S, double* out, int64_t cap, int64_t* n) {
    if (!S) return DIVAS_ERR_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    int64_t k = std::min<int64_t>(cap, (int64_t)S->lat_ms.size());
    for (int64_t i = 0; i < k && out; ++i) out[i] = S->lat_ms[i];
    if (n) *n = (int64_t)S->lat_ms.size();
    return DIVAS_OK;
}

divas_status divas_server_destroy(divas_server S) {
    if (!S) return DIVAS_ERR_ARG;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    S->th.join();
    for (auto& kv : S->sess)
        if (kv.second.s) (void)divas_session_destroy(kv.second.s);
    for (auto& sl : S->slots) {
        (void)hipStreamSynchronize(sl.st);
        (void)divas_batch_destroy(sl.b);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.st);
    }
    (void)hipStreamDestroy(S->admin);
    delete S;
    return DIVAS_OK;
}

}  // extern "C"
