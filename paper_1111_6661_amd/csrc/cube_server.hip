// cube_server.hip -- a query server over cubes resident in GPU memory.
//
// The paper offers its analysis as a service to many users, handling both
// batched and real-time requests (Abstract, Section 3), with a scheduler
// that allocates tasks from the status the workers publish (Section 2).  On
// one GPU that becomes a continuous-batching server: callers submit queries
// (statistics, histograms, fused or two-pass, over whole cubes or strided
// sub-boxes) from any thread; a worker thread forms batches with the policy
// of cube_policy.h and launches each batch on a free slot (a stream with its
// own persistent-launch batch object), so batches overlap on the device and
// new arrivals are admitted as soon as a slot and memory are free.  The
// worker observes completion through events and records each query's
// latency from submission to completion.
//
// The plain mode is the baseline a service without batching would use: one
// query at a time, in arrival order, each through the single-box entry
// point on one stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cube_internal.h"
#include "cube_policy.h"

using namespace cube;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Entry {
    cube_query_t q;
    double t_submit = 0, t_start = 0, t_done = 0;
    int state = 0;  // 0 waiting, 1 running, 2 done
    int rc = CUBE_OK;
    char err[160] = {0};
};

struct Slot {
    hipStream_t stream = nullptr;
    cube_batch_t *batch = nullptr;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> ids;
    bool busy = false;
    bool inject_event_error = false;  // test knob: this launch's event reports an error
};

int64_t query_voxels(const cube_query_t &q)
{
    if (q.dims[0] <= 0 || q.dims[1] <= 0 || q.dims[2] <= 0) return 0;
    return q.dims[0] * q.dims[1] * q.dims[2];
}

// Device scratch a query holds while in flight: its wavefront records
// (16 per 2^20 voxels, one tile each, two phases at most) and histogram
// accumulators.
int64_t query_scratch(const cube_query_t &q)
{
    const int64_t tiles = query_voxels(q) / (1 << 20) + 1;
    const int64_t bins = q.kind == CUBE_Q_STATS ? 0 : q.nbins;
    return tiles * 2 * 16 * 64 + bins * 8 + 256;
}

}  // namespace

struct cube_server {
    int mode = 0;  // 0 batched, 1 plain
    PolicyLimits lim;
    Policy *policy = nullptr;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    int device = 0;
    uint64_t next_id = 1;
    std::unordered_map<uint64_t, Entry> entries;
    std::vector<double> latencies;  // seconds, completed queries
    uint64_t n_done = 0, n_failed = 0;
    int64_t tile_voxels = 0;             // 0: each query's own automatic size
    uint64_t launches = 0;               // batches (or plain queries) launched
    std::vector<uint64_t> inject_fail;   // launch numbers that fail on purpose
    std::vector<uint64_t> inject_event;  // launch numbers whose event reports an error
};

namespace {

// Launch one batch (or one plain query) on a slot.  Called with the lock
// held.  Returns CUBE_OK or the first error (then no work was queued).
// Test knobs (CUBE_FAULT_INJECT, launches counted from 1 per server):
// "launch:N" makes launch N fail on the host before anything is queued, as
// a failed launch would; "event:N" makes the completion event of launch N
// report an error, as a device-side fault would (the work itself still runs
// to its end, so no kernel is affected).
int launch_on(cube_server *srv, Slot &sl, const std::vector<PolicyQuery> &batch)
{
    const uint64_t nth = ++srv->launches;
    for (uint64_t f : srv->inject_fail)
        if (f == nth)
            return fail(CUBE_EDEVICE, "injected launch failure (launch %llu)",
                        (unsigned long long)nth);
    sl.inject_event_error = false;
    for (uint64_t f : srv->inject_event)
        if (f == nth) sl.inject_event_error = true;
    std::vector<cube_query_t> qs;
    qs.reserve(batch.size());
    for (const PolicyQuery &p : batch) qs.push_back(srv->entries[p.id].q);
    int rc;
    if (srv->mode == 1) {
        const cube_query_t &q = qs[0];
        switch (q.kind) {
        case CUBE_Q_STATS: rc = cube_stats_async(q.ptr, q.dims, q.out, sl.stream); break;
        case CUBE_Q_HIST:
            rc = cube_hist_async(q.ptr, q.dims, q.lo, q.hi, q.nbins, q.counts, sl.stream);
            break;
        case CUBE_Q_FUSED:
            rc = cube_stats_hist_async(q.ptr, q.dims, q.lo, q.hi, q.nbins, q.out, q.counts,
                                       sl.stream);
            break;
        default:
            rc = cube_stats_hist_minmax_async(q.ptr, q.dims, q.nbins, q.out, q.counts, sl.stream);
        }
    } else {
        rc = cube_batch_enqueue(sl.batch, qs.data(), (int32_t)qs.size(), sl.stream);
    }
    if (rc) return rc;
    hipError_t e = hipEventRecord(sl.done, sl.stream);
    return e == hipSuccess ? CUBE_OK : hip_fail(e, "event record");
}

void worker_loop(cube_server *srv)
{
    hipSetDevice(srv->device);
    std::vector<PolicyQuery> batch;
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        // Completions: single queries as soon as their flags say so (the
        // batched mode), whole slots when their event has passed.
        bool any_done = false;
        for (int s = 0; s < (int)srv->slots.size(); ++s) {
            Slot &sl = srv->slots[s];
            if (!sl.busy) continue;
            const double t = now_s();
            // A query already completed may also have been collected (and
            // erased) by cube_server_wait: look entries up, never create.
            // Successes complete as soon as their flag is up; a failed query
            // is reported only once its whole launch has ended (below), so
            // its caller never frees outputs a kernel still writes.
            if (srv->mode == 0 && !sl.inject_event_error) {
                for (size_t k = 0; k < sl.ids.size(); ++k) {
                    auto it = srv->entries.find(sl.ids[k]);
                    if (it == srv->entries.end()) continue;
                    Entry &e = it->second;
                    if (e.state == 1 && cube_batch_query_done(sl.batch, (int32_t)k) == 1) {
                        e.state = 2;
                        e.t_done = t;
                        srv->latencies.push_back(t - e.t_submit);
                        ++srv->n_done;
                        any_done = true;
                    }
                }
            }
            hipError_t eq = sl.inject_event_error ? hipErrorLaunchFailure : hipEventQuery(sl.done);
            if (eq == hipErrorNotReady) continue;
            if (eq != hipSuccess) {
                // The launch failed on the device: its unfinished queries fail.
                // Wait for whatever still runs on the stream before the slot
                // is used again (a real fault returns at once).
                char msg[160];
                snprintf(msg, sizeof msg, "the launch of this query failed on the device: %s (%d)",
                         hipGetErrorString(eq), (int)eq);
                (void)hipGetLastError();
                lk.unlock();
                hipStreamSynchronize(sl.stream);
                (void)hipGetLastError();
                lk.lock();
                sl.inject_event_error = false;
                for (uint64_t id : sl.ids) {
                    auto it = srv->entries.find(id);
                    if (it == srv->entries.end()) continue;
                    Entry &e = it->second;
                    if (e.state == 2) continue;
                    e.state = 2;
                    e.rc = CUBE_EDEVICE;
                    e.t_done = now_s();
                    strncpy(e.err, msg, sizeof e.err - 1);
                    ++srv->n_failed;
                }
            } else {
                for (size_t k = 0; k < sl.ids.size(); ++k) {
                    auto it = srv->entries.find(sl.ids[k]);
                    if (it == srv->entries.end()) continue;
                    Entry &e = it->second;
                    if (e.state == 2) continue;
                    e.state = 2;
                    e.t_done = t;
                    // The launch has ended: a query whose flag says it failed
                    // (its range wait expired) reports that; the others are done.
                    if (srv->mode == 0 && cube_batch_query_done(sl.batch, (int32_t)k) < 0) {
                        e.rc = CUBE_EDEVICE;
                        strncpy(e.err, cube_last_error(), sizeof e.err - 1);
                        ++srv->n_failed;
                    } else {
                        srv->latencies.push_back(t - e.t_submit);
                        ++srv->n_done;
                    }
                }
            }
            sl.ids.clear();
            sl.busy = false;
            srv->policy->complete(s);
            any_done = true;
        }
        if (any_done) srv->cv_done.notify_all();
        // New batches on free slots.
        int slot;
        while ((slot = srv->policy->next_batch(batch)) >= 0) {
            Slot &sl = srv->slots[slot];
            const double t = now_s();
            const int rc = launch_on(srv, sl, batch);
            if (rc) {
                // The whole batch fails (the queries were validated on
                // submission, so this is a device-side error).
                for (const PolicyQuery &p : batch) {
                    Entry &e = srv->entries[p.id];
                    e.state = 2;
                    e.rc = rc;
                    e.t_done = t;
                    strncpy(e.err, cube_last_error(), sizeof e.err - 1);
                    ++srv->n_failed;
                }
                srv->policy->complete(slot);
                srv->cv_done.notify_all();
                continue;
            }
            for (const PolicyQuery &p : batch) {
                Entry &e = srv->entries[p.id];
                e.state = 1;
                e.t_start = t;
                sl.ids.push_back(p.id);
            }
            sl.busy = true;
        }
        if (srv->stop && srv->policy->busy_slots() == 0 && srv->policy->waiting() == 0) break;
        if (srv->policy->busy_slots() == 0 && srv->policy->waiting() == 0) {
            srv->cv_work.wait(lk);
        } else {
            // Work is in flight: poll its events again shortly.
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(10));
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

int cube_server_create(int32_t mode, int32_t slots, int32_t max_batch, int64_t max_inflight_bytes,
                       int64_t tile_voxels, cube_server_t **out)
{
    CUBE_GUARD_BEGIN
    if (!out) return fail(CUBE_EINVAL, "out is NULL");
    if (mode != CUBE_SERVE_BATCHED && mode != CUBE_SERVE_PLAIN)
        return fail(CUBE_EINVAL, "unknown server mode %d", mode);
    if (slots < 1 || slots > 16) return fail(CUBE_EINVAL, "slots outside [1, 16]");
    if (max_batch < 1 || max_batch > 4096) return fail(CUBE_EINVAL, "max_batch outside [1, 4096]");
    if (max_inflight_bytes < 4096) return fail(CUBE_EINVAL, "max_inflight_bytes too small");
    if (tile_voxels != 0 && (tile_voxels < 4096 || tile_voxels > ((int64_t)1 << 30)))
        return fail(CUBE_EINVAL, "tile_voxels outside [4096, 2^30]");
    cube_server *srv = new cube_server;
    srv->mode = mode == CUBE_SERVE_PLAIN ? 1 : 0;
    srv->lim.slots = srv->mode == 1 ? 1 : slots;
    srv->lim.max_batch = srv->mode == 1 ? 1 : max_batch;
    srv->lim.max_inflight_bytes = max_inflight_bytes;
    // About 2.5 ms of work per batch at the MI355X's streaming rate: a batch
    // never holds a slot much longer than one large query would.
    srv->lim.max_batch_voxels = (int64_t)1 << 32;
    if (tile_voxels) srv->tile_voxels = tile_voxels;
    srv->policy = new Policy(srv->lim);
    srv->inject_fail = fault_inject("launch");
    srv->inject_event = fault_inject("event");
    hipGetDevice(&srv->device);
    srv->slots.resize((size_t)srv->lim.slots);
    for (Slot &sl : srv->slots) {
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
            cube_server_destroy(srv);
            return hip_fail(e, "server slot");
        }
        int rc = cube_batch_create(&sl.batch);
        if (!rc) rc = cube_batch_set_tile(sl.batch, srv->tile_voxels, 0);
        if (!rc) rc = cube_batch_set_order(sl.batch, CUBE_ORDER_SMALLEST_FIRST);
        if (rc) {
            cube_server_destroy(srv);
            return rc;
        }
    }
    srv->worker = std::thread(worker_loop, srv);
    *out = srv;
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_server_submit(cube_server_t *srv, const cube_query_t *q, uint64_t *id)
{
    CUBE_GUARD_BEGIN
    if (!srv || !q || !id) return fail(CUBE_EINVAL, "NULL argument");
    // Host-side validation now; device-side checks happen at launch.
    Box box;
    int rc = check_box(q->ptr, q->dims, &box);
    if (rc) return rc;
    if (q->kind < CUBE_Q_STATS || q->kind > CUBE_Q_MINMAX)
        return fail(CUBE_EINVAL, "unknown query kind %d", q->kind);
    if (q->kind != CUBE_Q_STATS) {
        if (q->nbins < 1 || q->nbins > 32768) return fail(CUBE_EINVAL, "nbins outside [1, 32768]");
        HistRange r;
        if ((q->kind == CUBE_Q_HIST || q->kind == CUBE_Q_FUSED) &&
            (rc = check_range(q->lo, q->hi, q->nbins, &r)))
            return rc;
        if (!q->counts) return fail(CUBE_EINVAL, "counts is NULL");
    }
    if (q->kind != CUBE_Q_HIST && !q->out) return fail(CUBE_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(CUBE_EBUSY, "server is shutting down");
    const uint64_t k = srv->next_id++;
    PolicyQuery pq = {k, query_voxels(*q), query_scratch(*q)};
    if (!srv->policy->submit(pq)) return fail(CUBE_EBUSY, "queue full");
    Entry &e = srv->entries[k];
    e.q = *q;
    e.t_submit = now_s();
    *id = k;
    srv->cv_work.notify_one();
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_server_wait(cube_server_t *srv, uint64_t id, double timeout_s, double *latency_s)
{
    CUBE_GUARD_BEGIN
    if (!srv) return fail(CUBE_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->entries.find(id);
    if (it == srv->entries.end()) return fail(CUBE_EINVAL, "unknown query id %llu",
                                             (unsigned long long)id);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s));
    while (it->second.state != 2) {
        if (srv->cv_done.wait_until(lk, deadline) == std::cv_status::timeout &&
            it->second.state != 2)
            return fail(CUBE_EBUSY, "query %llu not done within %.3f s", (unsigned long long)id,
                        timeout_s);
        it = srv->entries.find(id);
    }
    const Entry e = it->second;
    srv->entries.erase(it);
    if (latency_s) *latency_s = e.t_done - e.t_submit;
    if (e.rc) return fail(e.rc, "%s", e.err);
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_server_latency(cube_server_t *srv, double *p50_s, double *p99_s, uint64_t *n_done,
                        int32_t reset)
{
    CUBE_GUARD_BEGIN
    if (!srv) return fail(CUBE_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    std::vector<double> v = srv->latencies;
    if (n_done) *n_done = v.size();
    double p50 = NAN, p99 = NAN;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double idx = p * (double)(v.size() - 1);
            const size_t lo = (size_t)floor(idx), hi = (size_t)ceil(idx);
            return v[lo] + (v[hi] - v[lo]) * (idx - (double)lo);
        };
        p50 = pct(0.50);
        p99 = pct(0.99);
    }
    if (p50_s) *p50_s = p50;
    if (p99_s) *p99_s = p99;
    if (reset) srv->latencies.clear();
    return CUBE_OK;
    CUBE_GUARD_END
}

void cube_server_destroy(cube_server_t *srv)
{
    CUBE_GUARD_BEGIN
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (Slot &sl : srv->slots) {
        if (sl.stream) hipStreamSynchronize(sl.stream);
        if (sl.batch) cube_batch_destroy(sl.batch);
        if (sl.done) hipEventDestroy(sl.done);
        if (sl.stream) {
            release_ws(sl.stream);  // the plain mode's single-box workspace
            hipStreamDestroy(sl.stream);
        }
    }
    delete srv->policy;
    delete srv;
    CUBE_GUARD_VOID_END
}

}  // extern "C"
