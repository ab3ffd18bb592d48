// Decode server: continuous batching of decode requests under an HBM budget.
//
// Requests are device-resident streams (words, gap array, chunk offsets,
// table).  The server owns one device arena of `hbm_budget` bytes from which
// it allocates every admitted request's output and each multi-request
// batch's workspace, so the in-flight footprint never exceeds the budget.  A
// scheduler thread loops: it retires batches whose completion event has
// fired, then admits queued requests in arrival order while their output
// fits in the arena (head-of-line: a request that does not fit waits for
// memory to free), and launches each admitted group on a free HIP stream --
// a lone request as the one-launch gap-mode decode, several as one batched
// launch -- outside the lock, so submit, poll and release never wait for a
// launch.  Each stream slot's status word lives in pinned host memory: the
// host zeroes it before the launch and the kernels store nonzero error bits
// into it, so no copy follows the decode.  While batches run (and for a short
// idle window) the scheduler polls their events instead of sleeping; after
// that it blocks until a submit or release.  Requests arriving while earlier
// batches run are admitted into new batches on other streams, so their work
// overlaps on the device.  Outputs stay allocated until the client releases
// them.  Destroying the server waits for running batches and drops requests
// that were never admitted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hd.h"
#include "hd_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_s()
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte granules.
class Arena {
public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }

    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) / 256 * 256;
        if (bytes == 0)
            bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                used_ += bytes;
                sizes_[*off] = bytes;
                return true;
            }
        }
        return false;
    }

    void release(size_t off)
    {
        auto s = sizes_.find(off);
        if (s == sizes_.end())
            return;
        size_t len = s->second;
        sizes_.erase(s);
        used_ -= len;
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        auto prev = free_.lower_bound(off);
        if (prev != free_.begin()) {
            --prev;
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }

    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;             // offset -> length
    std::unordered_map<size_t, size_t> sizes_;  // allocated offset -> length
};

enum class ReqState { Queued, Running, Done };

struct Request {
    uint64_t id;
    hd_dstream s;
    size_t out_off = 0;
    ReqState state = ReqState::Queued;
    hd_status status = HD_OK;
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Batch {
    std::vector<uint64_t> ids;
    std::vector<hd_dstream> ds;          // copies taken under the lock, launched outside it
    std::vector<uint16_t *> outs;
    size_t ws_off = 0, ws_bytes = 0;     // a batch workspace (several requests only)
    bool has_ws = false;
    int slot = -1;
    hipEvent_t done = nullptr;
    hd_status launch_status = HD_OK;
};

// Busy-poll window of an idle scheduler before it blocks on the condition
// variable (a blocked thread takes a futex wake-up, tens of microseconds, to
// see the next submit).
constexpr auto kIdleSpin = std::chrono::milliseconds(50);

}  // namespace

struct hd_server {
    int device = 0;
    uint32_t max_batch = 64;
    void *base = nullptr;
    Arena *arena = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<bool> slot_busy;
    // pinned, one status word per stream slot: zeroed by the host before a
    // launch, written by the decode kernels (no copy after the decode)
    volatile uint32_t *status_host = nullptr;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<uint64_t> done_q;
    std::vector<Batch> running;          // touched by the scheduler thread only
    uint64_t next_id = 1;
    std::atomic<bool> stop{false};
    std::atomic<uint64_t> epoch{0};      // bumped by submit and release (under mu)
    std::thread worker;
    uint64_t n_batches = 0, n_done = 0, peak_used = 0;

    void loop();
    void retire_locked();
    void admit_locked(std::vector<Batch> &out);
    void launch(Batch &b);
    void finish_locked(Batch &b);
    void wait_for_change(uint64_t seen, Clock::time_point idle_since);
};

void hd_server::retire_locked()
{
    for (size_t b = 0; b < running.size();) {
        Batch &bt = running[b];
        const hipError_t q = hipEventQuery(bt.done);
        if (q == hipErrorNotReady) {
            ++b;
            continue;
        }
        // completed, or the device reported an error for this stream
        const double t = now_s();
        const hd_status st = q != hipSuccess ? HD_ERR_DEVICE : status_host[bt.slot] ? HD_ERR_CORRUPT : HD_OK;
        for (uint64_t id : bt.ids) {
            Request &r = reqs[id];
            r.state = ReqState::Done;
            r.t_done = t;
            r.status = st;
            done_q.push_back(id);
            ++n_done;
        }
        if (bt.has_ws)
            arena->release(bt.ws_off);
        slot_busy[bt.slot] = false;
        running.erase(running.begin() + b);
    }
}

// Admits queued requests in arrival order into batches, one per free stream
// slot: outputs (and, for several requests, the batch workspace) come from
// the arena; a request that does not fit waits at the head of the queue.
void hd_server::admit_locked(std::vector<Batch> &out)
{
    for (;;) {
        if (queue.empty())
            return;
        int slot = -1;
        for (size_t i = 0; i < slot_busy.size(); ++i)
            if (!slot_busy[i]) {
                slot = static_cast<int>(i);
                break;
            }
        if (slot < 0)
            return;
        std::vector<uint64_t> ids;
        while (!queue.empty() && ids.size() < max_batch) {
            Request &r = reqs[queue.front()];
            size_t off = 0;
            if (!arena->alloc(r.s.info.n_symbols * 2 + 16, &off))
                break;
            r.out_off = off;
            ids.push_back(queue.front());
            queue.pop_front();
        }
        if (ids.empty())
            return;
        Batch bt;
        // several requests share one batched launch and its workspace; shrink
        // the batch until the workspace fits (one request needs none)
        for (;;) {
            bt.ds.resize(ids.size());
            bt.outs.resize(ids.size());
            for (size_t i = 0; i < ids.size(); ++i) {
                bt.ds[i] = reqs[ids[i]].s;
                bt.outs[i] = reinterpret_cast<uint16_t *>(static_cast<char *>(base) + reqs[ids[i]].out_off);
            }
            if (ids.size() == 1)
                break;
            size_t wsb = 0;
            if (hd_decode_batch_workspace_size(bt.ds.data(), static_cast<uint32_t>(bt.ds.size()), HD_MODE_GAP,
                                               &wsb) == HD_OK &&
                arena->alloc(wsb, &bt.ws_off)) {
                bt.ws_bytes = wsb;
                bt.has_ws = true;
                break;
            }
            arena->release(reqs[ids.back()].out_off);
            queue.push_front(ids.back());
            ids.pop_back();
        }
        const double t = now_s();
        for (uint64_t id : ids) {
            reqs[id].state = ReqState::Running;
            reqs[id].t_start = t;
        }
        bt.ids = std::move(ids);
        bt.slot = slot;
        bt.done = events[slot];
        slot_busy[slot] = true;
        peak_used = std::max<uint64_t>(peak_used, arena->used());
        out.push_back(std::move(bt));
    }
}

// Enqueues one batch on its stream slot (outside the lock): a single request
// takes the one-launch gap-mode decode, several take one batched launch.
void hd_server::launch(Batch &bt)
{
    status_host[bt.slot] = 0;
    hipStream_t st = streams[bt.slot];
    uint32_t *sw = const_cast<uint32_t *>(&status_host[bt.slot]);
    hd_status r = bt.ds.size() == 1
                      ? hd::decode_gap_direct(&bt.ds[0], bt.outs[0], sw, st)
                      : hd::decode_batch_direct(bt.ds.data(), static_cast<uint32_t>(bt.ds.size()), bt.outs.data(),
                                                sw, static_cast<char *>(base) + bt.ws_off, bt.ws_bytes, st);
    if (r == HD_OK && hipEventRecord(bt.done, st) != hipSuccess) {
        (void)hipStreamSynchronize(st);      // the decode may still use the workspace
        r = HD_ERR_DEVICE;
    }
    bt.launch_status = r;
}

void hd_server::finish_locked(Batch &bt)
{
    if (bt.launch_status == HD_OK) {
        running.push_back(std::move(bt));
        ++n_batches;
        return;
    }
    const double t = now_s();
    for (uint64_t id : bt.ids) {
        Request &r = reqs[id];
        r.state = ReqState::Done;
        r.status = bt.launch_status;
        r.t_done = t;
        done_q.push_back(id);
        ++n_done;
    }
    if (bt.has_ws)
        arena->release(bt.ws_off);
    slot_busy[bt.slot] = false;
}

// Returns once something may have changed: a submit or release (epoch), a
// running batch's event, or stop.  Polls while batches run or for a short
// idle window, then blocks on the condition variable.
void hd_server::wait_for_change(uint64_t seen, Clock::time_point idle_since)
{
    for (;;) {
        if (stop.load(std::memory_order_acquire) || epoch.load(std::memory_order_acquire) != seen)
            return;
        for (const Batch &b : running)
            if (hipEventQuery(b.done) != hipErrorNotReady)
                return;
        if (running.empty() && Clock::now() - idle_since > kIdleSpin) {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop.load() || epoch.load() != seen; });
            return;
        }
        std::this_thread::yield();
    }
}

void hd_server::loop()
{
    (void)hipSetDevice(device);
    Clock::time_point idle_since = Clock::now();
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        retire_locked();
        if (stop.load() && running.empty())
            break;
        std::vector<Batch> ls;
        if (!stop.load())
            admit_locked(ls);
        if (!ls.empty()) {
            lk.unlock();                     // submit, poll and release go on meanwhile
            for (Batch &b : ls)
                launch(b);
            lk.lock();
            for (Batch &b : ls)
                finish_locked(b);
            idle_since = Clock::now();
            continue;
        }
        if (!running.empty())
            idle_since = Clock::now();
        const uint64_t seen = epoch.load();
        lk.unlock();
        wait_for_change(seen, idle_since);
        lk.lock();
    }
}

extern "C" hd_status hd_server_create(size_t hbm_budget, uint32_t n_hip_streams, uint32_t max_batch,
                                      hd_server **out)
{
    if (!out || hbm_budget < 4096 || n_hip_streams == 0 || n_hip_streams > 64 || max_batch == 0)
        return HD_ERR_ARG;
    *out = nullptr;
    hd_server *s = new (std::nothrow) hd_server();
    if (!s)
        return HD_ERR_NOMEM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return HD_ERR_DEVICE;
    }
    s->max_batch = max_batch;
    if (hipMalloc(&s->base, hbm_budget) != hipSuccess) {
        delete s;
        return HD_ERR_NOMEM;
    }
    s->arena = new Arena(hbm_budget);
    if (hipHostMalloc(const_cast<void **>(reinterpret_cast<volatile void **>(&s->status_host)),
                      sizeof(uint32_t) * n_hip_streams, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(s->base);
        delete s->arena;
        delete s;
        return HD_ERR_NOMEM;
    }
    for (uint32_t i = 0; i < n_hip_streams; ++i) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            for (auto x : s->streams)
                (void)hipStreamDestroy(x);
            for (auto x : s->events)
                (void)hipEventDestroy(x);
            (void)hipHostFree(const_cast<uint32_t *>(s->status_host));
            (void)hipFree(s->base);
            delete s->arena;
            delete s;
            return HD_ERR_DEVICE;
        }
        s->streams.push_back(st);
        s->events.push_back(ev);
        s->slot_busy.push_back(false);
    }
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return HD_OK;
}

extern "C" void hd_server_destroy(hd_server *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop.store(true);
    }
    s->cv.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto ev : s->events)
        (void)hipEventDestroy(ev);
    (void)hipHostFree(const_cast<uint32_t *>(s->status_host));
    (void)hipFree(s->base);
    delete s->arena;
    delete s;
}

extern "C" hd_status hd_server_submit(hd_server *s, const hd_dstream *stream, uint64_t *request_id)
{
    if (!s || !stream || !request_id)
        return HD_ERR_ARG;
    size_t wsb = 0;
    hd_status st = hd_decode_batch_workspace_size(stream, 1, HD_MODE_GAP, &wsb);
    if (st != HD_OK)
        return st;
    const size_t need = (stream->info.n_symbols * 2 + 16 + 255) / 256 * 256 + (wsb + 255) / 256 * 256;
    std::lock_guard<std::mutex> lk(s->mu);
    if (need > s->arena->size())
        return HD_ERR_NOMEM;                 // can never be admitted under this budget
    Request r;
    r.id = s->next_id++;
    r.s = *stream;
    r.t_submit = now_s();
    s->reqs.emplace(r.id, r);
    s->queue.push_back(r.id);
    *request_id = r.id;
    s->epoch.fetch_add(1, std::memory_order_release);
    s->cv.notify_all();
    return HD_OK;
}

extern "C" hd_status hd_server_poll(hd_server *s, uint64_t *done_ids, uint32_t cap, uint32_t *n_done)
{
    if (!s || !n_done || (cap && !done_ids))
        return HD_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t k = 0;
    while (k < cap && !s->done_q.empty()) {
        done_ids[k++] = s->done_q.front();
        s->done_q.pop_front();
    }
    *n_done = k;
    return HD_OK;
}

extern "C" hd_status hd_server_result(hd_server *s, uint64_t id, const uint16_t **out, hd_status *status,
                                      double *t_submit, double *t_done)
{
    if (!s)
        return HD_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second.state != ReqState::Done)
        return HD_ERR_ARG;
    const Request &r = it->second;
    if (out)
        *out = reinterpret_cast<const uint16_t *>(static_cast<const char *>(s->base) + r.out_off);
    if (status)
        *status = r.status;
    if (t_submit)
        *t_submit = r.t_submit;
    if (t_done)
        *t_done = r.t_done;
    return HD_OK;
}

extern "C" hd_status hd_server_release(hd_server *s, uint64_t id)
{
    if (!s)
        return HD_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second.state != ReqState::Done)
        return HD_ERR_ARG;
    s->arena->release(it->second.out_off);
    s->reqs.erase(it);
    s->epoch.fetch_add(1, std::memory_order_release);
    s->cv.notify_all();
    return HD_OK;
}

extern "C" hd_status hd_server_stats(hd_server *s, uint64_t *n_batches, uint64_t *n_done, uint64_t *queued,
                                     uint64_t *arena_used, uint64_t *arena_peak)
{
    if (!s)
        return HD_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (n_batches)
        *n_batches = s->n_batches;
    if (n_done)
        *n_done = s->n_done;
    if (queued)
        *queued = s->queue.size();
    if (arena_used)
        *arena_used = s->arena->used();
    if (arena_peak)
        *arena_peak = s->peak_used;
    return HD_OK;
}
