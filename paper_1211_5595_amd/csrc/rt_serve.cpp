// rt_serve.cpp -- the serving runtime behind include/rt_serve.h: a request
// queue, admission against an image pool, continuous batching onto a few
// streams that replay captured batch plans, and a server thread that uploads
// tables, launches and retires batches.  See rt_serve.h for the contract.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rt.h"
#include "rt_internal.h"
#include "rt_serve.h"

using namespace rtv;

namespace {

constexpr int kMaxStreams = 8;
constexpr int kMaxServerBatch = 256;

size_t r256(size_t x) { return (x + 255) & ~(size_t)255; }

double now_s() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

rt_status err(rt_status s, const std::string& m) { return static_cast<rt_status>(set_last_error(s, m.c_str())); }

size_t slot_bytes() {
    size_t b = 0;
    rt_tf_bytes(kMaxK, &b);
    return r256(b);
}
size_t workspace_bytes(int max_batch) {
    size_t b = 0;
    rt_batch_workspace_bytes(max_batch, &b);
    return r256(b);
}
// Per stream: workspace, max_batch table slots.
size_t lane_bytes(int max_batch) { return workspace_bytes(max_batch) + (size_t)max_batch * slot_bytes(); }

// First-fit allocator over [0, size) with coalescing; offsets 256-aligned.
struct Pool {
    size_t size = 0, in_use = 0, peak = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t n) {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            in_use += n;
            peak = std::max(peak, in_use);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        in_use -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
};

struct Req {
    rt_request r;
    std::vector<float> table;
    const float* ext_table = nullptr;  // the caller's table, while rt_server_submit launches the request itself
    rt_request_info info;
    size_t img_off = 0, img_bytes = 0;
    bool has_img = false;
};

struct Slot {
    void* dev = nullptr;
    rt_tf* tf = nullptr;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    rt_batch_plan* plan = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<Slot> slots;
    std::vector<uint64_t> tickets;
    bool busy = false;
    bool launching = false;  // busy, and its launch still being enqueued (the event is not yet this batch's)
};

}  // namespace

struct rt_server {
    int device = 0;
    int max_batch = 0;
    long long batch_pixels = 0;  // a batch closes before it would exceed this many pixels
    int kind = -1;
    int skip = 0;
    unsigned long long* counter = nullptr;  // caller's device sample counter, nullable
    char* pool_base = nullptr;
    Pool pool;
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    uint64_t next_ticket = 0;
    bool stop = false;
    rt_server_stats stats{};
    std::thread thread;

    void loop();
    bool retire_locked();
    bool launch(std::unique_lock<std::mutex>& lk);
};

// Retire finished batches (lock held).
bool rt_server::retire_locked() {
    bool any = false;
    for (size_t k = 0; k < lanes.size(); ++k) {
        Lane& L = lanes[k];
        if (!L.busy || L.launching) continue;
        const hipError_t e = hipEventQuery(L.done);
        if (e == hipErrorNotReady) continue;
        const double t = now_s();
        for (uint64_t id : L.tickets) {
            Req& q = reqs.at(id);
            q.info.t_done = t;
            q.info.batch_size = (int)L.tickets.size();
            if (e == hipSuccess) {
                q.info.state = RT_REQ_DONE;
                q.info.image_dev = reinterpret_cast<float*>(pool_base + q.img_off);
                ++stats.completed;
            } else {
                q.info.state = RT_REQ_FAILED;
                q.info.status = RT_ERR_DEVICE;
                pool.release(q.img_off, q.img_bytes);
                q.has_img = false;
                ++stats.failed;
            }
        }
        stats.running -= (int)L.tickets.size();
        L.tickets.clear();
        L.busy = false;
        any = true;
    }
    if (any) cv_done.notify_all();
    return any;
}

// Admit the head of the queue into one free lane and launch it.  Called with
// the lock held; drops it around the uploads and the launch.
bool rt_server::launch(std::unique_lock<std::mutex>& lk) {
    if (queue.empty()) return false;
    int k = -1;
    for (size_t i = 0; i < lanes.size(); ++i)
        if (!lanes[i].busy) {
            k = (int)i;
            break;
        }
    if (k < 0) return false;
    Lane& L = lanes[k];
    std::vector<uint64_t> batch;
    long long pixels = 0;
    while (!queue.empty() && (int)batch.size() < max_batch) {
        Req& q = reqs.at(queue.front());
        const long long px = (long long)q.r.width * q.r.height;
        if (!batch.empty() && pixels + px > batch_pixels) break;  // the rest goes to the next free stream
        size_t off;
        if (!pool.alloc(q.img_bytes, &off)) break;  // the head waits for memory
        q.img_off = off;
        q.has_img = true;
        q.info.state = RT_REQ_RUNNING;
        batch.push_back(queue.front());
        queue.pop_front();
        pixels += px;
    }
    if (batch.empty()) return false;
    L.busy = true;  // reserved while unlocked
    L.launching = true;
    L.tickets = batch;
    stats.queued -= (int)batch.size();
    stats.running += (int)batch.size();
    // stamped as the batch leaves the queue (under the lock, so in queue order
    // whichever thread launches it)
    const double t_launch = now_s();
    std::vector<Req*> rq;
    for (uint64_t id : batch) {
        rq.push_back(&reqs.at(id));  // stable: queued/running requests are never erased
        rq.back()->info.t_launch = t_launch;
    }
    lk.unlock();

    rt_status st = RT_OK;
    std::vector<rt_render_job> jobs(batch.size());
    for (size_t j = 0; j < batch.size() && st == RT_OK; ++j) {
        Req& q = *rq[j];
        Slot& sl = L.slots[j];  // created with 4096 entries: any table fits, nothing is allocated here
        st = rt_set_transfer_function(&sl.tf, q.ext_table ? q.ext_table : q.table.data(), q.r.tf_entries,
                                      q.r.tf_vmin, q.r.tf_vmax, sl.dev, slot_bytes(), L.stream);
        if (st != RT_OK) break;
        rt_render_job& J = jobs[j];
        std::memset(&J, 0, sizeof(J));
        J.volume = q.r.volume;
        J.tf = sl.tf;
        J.camera = q.r.camera;
        J.width = q.r.width;
        J.height = q.r.height;
        J.step_vox = q.r.step_vox;
        J.alpha_cutoff = q.r.alpha_cutoff;
        for (int c = 0; c < 4; ++c) J.bg_rgba[c] = q.r.bg_rgba[c];
        J.out_dev = reinterpret_cast<float*>(pool_base + q.img_off);
        J.pixel_counts = nullptr;
        J.ray_function = q.r.ray_function;
        J.iso_value = q.r.iso_value;
        J.iso_high = q.r.iso_high;
        J.opacity_unit_distance = q.r.opacity_unit_distance;
        J.skip_empty = skip;
    }
    if (st == RT_OK) st = rt_batch_plan_launch(L.plan, jobs.data(), (int)jobs.size(), counter, L.stream);
    if (st == RT_OK && hipEventRecord(L.done, L.stream) != hipSuccess) st = RT_ERR_DEVICE;

    lk.lock();
    L.launching = false;
    ++stats.batches;
    if (st != RT_OK) {  // the batch never reached the device: fail its requests
        for (Req* q : rq) {
            q->info.state = RT_REQ_FAILED;
            q->info.status = st;
            q->info.t_done = now_s();
            pool.release(q->img_off, q->img_bytes);
            q->has_img = false;
            ++stats.failed;
        }
        stats.running -= (int)batch.size();
        L.tickets.clear();
        L.busy = false;
        cv_done.notify_all();
    }
    return true;
}

void rt_server::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = retire_locked();
        progressed = launch(lk) || progressed;
        bool busy = false;
        for (const Lane& L : lanes) busy = busy || L.busy;
        if (stop && !busy && !progressed && !queue.empty()) {
            // shutting down with nothing running and the head still not admitted:
            // the pool is held by unreleased requests, so the rest can never run
            const double t = now_s();
            for (uint64_t id : queue) {
                Req& q = reqs.at(id);
                q.info.state = RT_REQ_FAILED;
                q.info.status = RT_ERR_OUT_OF_MEMORY;
                q.info.t_done = t;
                ++stats.failed;
            }
            stats.queued -= (int)queue.size();
            queue.clear();
            cv_done.notify_all();
        }
        if (stop && queue.empty() && !busy) break;
        if (progressed) continue;
        if (busy) {  // completion is polled: yield, a timed sleep would add its granularity to every request
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            cv_work.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

namespace {

void destroy_resources(rt_server* s) {
    for (Lane& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        for (Slot& sl : L.slots)
            if (sl.tf) rt_destroy_tf(sl.tf);
        if (L.plan) rt_batch_plan_destroy(L.plan);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    delete s;
}

}  // namespace

extern "C" {

rt_status rt_server_arena_bytes(int n_streams, int max_batch, size_t image_pool_bytes, size_t* bytes) {
    if (!bytes) return err(RT_ERR_INVALID_ARG, "bytes is NULL");
    if (n_streams < 1 || n_streams > kMaxStreams) return err(RT_ERR_INVALID_ARG, "n_streams must be in [1, 8]");
    if (max_batch < 1 || max_batch > kMaxServerBatch) return err(RT_ERR_INVALID_ARG, "max_batch must be in [1, 256]");
    if (image_pool_bytes < 256) return err(RT_ERR_INVALID_ARG, "image pool must hold at least 256 bytes");
    *bytes = (size_t)n_streams * lane_bytes(max_batch) + r256(image_pool_bytes);
    return RT_OK;
}

rt_status rt_server_create(int n_streams, int max_batch, int storage, int layout, const rt_render_opts* opts,
                           void* arena_dev, size_t arena_bytes, size_t image_pool_bytes, rt_server** out) {
    if (!out) return err(RT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    rt_status st = rt_server_arena_bytes(n_streams, max_batch, image_pool_bytes, &need);
    if (st != RT_OK) return st;
    const int kind = storage_layout_kind(storage, layout);
    if (kind < 0) return err(RT_ERR_INVALID_ARG, "unknown storage type or layout not available for it");
    if (!arena_dev) return err(RT_ERR_INVALID_ARG, "arena is NULL");
    if (((uintptr_t)arena_dev & 255) != 0) return err(RT_ERR_INVALID_ARG, "arena must be 256-byte aligned");
    if (arena_bytes < need) return err(RT_ERR_OUT_OF_MEMORY, "arena smaller than rt_server_arena_bytes");
    if (opts && (opts->tile_order < 0 || opts->tile_order > 2)) return err(RT_ERR_INVALID_ARG, "tile_order must be 0, 1 or 2");

    rt_server* s = new (std::nothrow) rt_server;
    if (!s) return err(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
    (void)hipGetDevice(&s->device);
    s->max_batch = max_batch;
    // about 16 views' worth of the rays the GPU holds at once: near the
    // persistent launch's full throughput, and ~1 ms of work, so a burst is
    // split over the streams instead of completing as one long batch
    s->batch_pixels = 16 * rt_batch_latency_pixels();
    s->kind = kind;
    s->skip = opts && opts->skip_empty ? 1 : 0;
    s->counter = opts ? opts->sample_counter : nullptr;
    rt_render_opts po;
    std::memset(&po, 0, sizeof(po));
    if (opts) {
        po.tile_w = opts->tile_w;
        po.tile_h = opts->tile_h;
        po.waves_per_block = opts->waves_per_block;
        po.skip_empty = opts->skip_empty;
        po.tile_order = opts->tile_order;
        po.batch_form = opts->batch_form;
    }
    hipError_t e = hipSuccess;
    char* base = static_cast<char*>(arena_dev);
    s->lanes.resize(n_streams);
    for (int k = 0; k < n_streams; ++k) {
        Lane& L = s->lanes[k];
        char* lb = base + (size_t)k * lane_bytes(max_batch);
        L.ws = lb;
        L.ws_bytes = workspace_bytes(max_batch);
        L.slots.resize(max_batch);
        for (int j = 0; j < max_batch; ++j) L.slots[j].dev = lb + L.ws_bytes + (size_t)j * slot_bytes();
        e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            destroy_resources(s);
            return err(RT_ERR_DEVICE, std::string("stream set-up: ") + hipGetErrorString(e));
        }
        st = rt_batch_plan_create(max_batch, storage, layout, L.ws, L.ws_bytes, &po, &L.plan);
        if (st != RT_OK) {
            const std::string m = rt_last_error();
            destroy_resources(s);
            return err(st, "batch plan: " + m);
        }
        // every table slot's handle (and its pinned staging buffer) made now,
        // at the largest size, so the request path never allocates or frees
        // pinned memory (calls that can wait for the whole device)
        const std::vector<float> blank(4 * (size_t)kMaxK, 0.0f);
        for (int j = 0; j < max_batch && st == RT_OK; ++j)
            st = rt_set_transfer_function(&L.slots[j].tf, blank.data(), kMaxK, 0.0, 1.0, L.slots[j].dev, slot_bytes(),
                                          L.stream);
        if (st != RT_OK) {
            const std::string m = rt_last_error();
            destroy_resources(s);
            return err(st, "table slots: " + m);
        }
        e = hipStreamSynchronize(L.stream);
        if (e != hipSuccess) {
            destroy_resources(s);
            return err(RT_ERR_DEVICE, std::string("stream set-up: ") + hipGetErrorString(e));
        }
    }
    s->pool_base = base + (size_t)n_streams * lane_bytes(max_batch);
    s->pool.init(r256(image_pool_bytes));
    s->stats.pool_bytes = s->pool.size;
    try {
        s->thread = std::thread([s] { s->loop(); });
    } catch (...) {
        destroy_resources(s);
        return err(RT_ERR_DEVICE, "could not start the server thread");
    }
    *out = s;
    return RT_OK;
}

rt_status rt_server_submit(rt_server* s, const rt_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return err(RT_ERR_INVALID_ARG, "NULL server, request or ticket");
    if (!req->tf_rgba) return err(RT_ERR_INVALID_ARG, "NULL table");
    const int K = req->tf_entries;
    int kind = -1;
    rt_status st = static_cast<rt_status>(check_request(req->volume, K, req->tf_vmin, req->tf_vmax, &req->camera,
                                                        req->width, req->height, req->step_vox, req->alpha_cutoff,
                                                        req->bg_rgba, reinterpret_cast<const float*>((uintptr_t)256),
                                                        req->ray_function, req->iso_value, req->iso_high,
                                                        req->opacity_unit_distance, &kind));
    if (st != RT_OK) return st;
    if (kind != s->kind) return err(RT_ERR_INVALID_ARG, "volume of another storage type or layout than the server's");
    if (!unit_range(req->tf_rgba, 4 * (size_t)K)) return err(RT_ERR_INVALID_ARG, "table entries must be in [0, 1]");
    const size_t img = r256((size_t)req->width * (size_t)req->height * 16);
    if (img > s->pool.size) return err(RT_ERR_OUT_OF_MEMORY, "image larger than the server's image pool");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop) return err(RT_ERR_INVALID_ARG, "server is shutting down");
    const uint64_t id = ++s->next_ticket;
    Req& q = s->reqs[id];
    q.r = *req;
    q.r.tf_rgba = nullptr;
    std::memset(&q.info, 0, sizeof(q.info));
    q.info.state = RT_REQ_QUEUED;
    q.info.status = RT_OK;
    q.info.t_submit = now_s();
    q.img_bytes = img;
    s->queue.push_back(id);
    ++s->stats.submitted;
    ++s->stats.queued;
    *ticket = id;
    // A request that finds the queue otherwise empty and a stream free is
    // launched from the caller's thread: the server thread would first have
    // to wake up.  Its table is uploaded from the caller's memory (the lock is
    // held from the push until launch() takes the queue's head, so no other
    // thread can take it).  The server thread retires it as any other batch.
    bool free_lane = false;
    if (s->queue.size() == 1)
        for (const Lane& L : s->lanes) free_lane = free_lane || !L.busy;
    if (free_lane) {
        q.ext_table = req->tf_rgba;
        int prev = -1;
        const bool other = hipGetDevice(&prev) == hipSuccess && prev != s->device;
        if (other) (void)hipSetDevice(s->device);
        s->launch(lk);
        if (other) (void)hipSetDevice(prev);
        q.ext_table = nullptr;  // uploaded, or still queued (then it gets its own copy below)
    }
    if (q.info.state == RT_REQ_QUEUED) q.table.assign(req->tf_rgba, req->tf_rgba + 4 * (size_t)K);
    s->cv_work.notify_one();
    return RT_OK;
}

rt_status rt_server_wait(rt_server* s, uint64_t ticket, double timeout_s, rt_request_info* info) {
    if (!s || !info) return err(RT_ERR_INVALID_ARG, "NULL server or info");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return err(RT_ERR_INVALID_ARG, "unknown ticket");
    auto finished = [&] {
        const int st = s->reqs.at(ticket).info.state;
        return st == RT_REQ_DONE || st == RT_REQ_FAILED;
    };
    if (timeout_s < 0.0)
        s->cv_done.wait(lk, finished);
    else if (timeout_s > 0.0)
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished);
    *info = s->reqs.at(ticket).info;
    return RT_OK;
}

rt_status rt_server_release(rt_server* s, uint64_t ticket) {
    if (!s) return err(RT_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return err(RT_ERR_INVALID_ARG, "unknown ticket");
    Req& q = it->second;
    if (q.info.state != RT_REQ_DONE && q.info.state != RT_REQ_FAILED)
        return err(RT_ERR_INVALID_ARG, "request still queued or running");
    if (q.has_img) s->pool.release(q.img_off, q.img_bytes);
    s->reqs.erase(it);
    s->cv_work.notify_one();  // memory came back: the head of the queue may fit now
    return RT_OK;
}

rt_status rt_server_get_stats(rt_server* s, rt_server_stats* out) {
    if (!s || !out) return err(RT_ERR_INVALID_ARG, "NULL server or stats");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->pool_in_use = s->pool.in_use;
    out->pool_peak = s->pool.peak;
    return RT_OK;
}

rt_status rt_server_destroy(rt_server* s) {
    if (!s) return RT_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_one();
    }
    if (s->thread.joinable()) s->thread.join();
    destroy_resources(s);
    return RT_OK;
}

}  // extern "C"
