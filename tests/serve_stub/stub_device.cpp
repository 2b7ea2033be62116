// Simulated device for the serving runtime's CPU concurrency test.  Test
// infrastructure only: rt_serve.cpp is compiled unchanged against the stub
// HIP header beside this file and linked with these stand-ins instead of the
// HIP runtime and the renderer, then run under ThreadSanitizer.
//
// A stream is an in-order queue of work items run by a worker thread of its
// own; an event is the stream's item count at record time, complete once the
// worker has finished that many items (release/acquire on the count, so what
// an item wrote is visible to whoever saw the event complete).  A "kernel"
// writes every pixel of every job's image (host memory standing in for the
// arena) from the job's size, camera and the first entry of the table slot
// the server uploaded on the same stream, after a short random pause; the
// driver checks each image against its own request.  Event fields are plain
// memory on purpose: only the server's own locking orders a record against a
// query made from another thread.
#include <hip/hip_runtime.h>
#include <pthread.h>
#include <time.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "rt.h"
#include "rt_internal.h"

struct StubStream {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> items;
    uint64_t submitted = 0;  // guarded by mu
    std::atomic<uint64_t> completed{0};
    bool stop = false;
    std::thread worker;
};

struct StubEvent {
    StubStream* stream = nullptr;
    uint64_t seq = 0;
};

struct rt_volume {
    int kind;
};

struct rt_tf {
    int K;
    int cap;     // entries the handle was created with
    float* dev;  // the table slot in the arena
};

struct rt_batch_plan {
    int max_jobs;
    int kind;
};

std::atomic<long> g_jobs_rendered{0};
std::atomic<int> g_max_pause_us{200};
std::atomic<long> g_max_multi_batch_pixels{0};  // the largest pixel total of a launch of two or more jobs

namespace {

thread_local int t_device = 0;
thread_local std::string t_error;

void enqueue(StubStream* s, std::function<void()> f) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->items.push_back(std::move(f));
        ++s->submitted;
    }
    s->cv.notify_all();
}

void worker_loop(StubStream* s) {
    std::mt19937 rng(reinterpret_cast<uintptr_t>(s) & 0xffffffffu);
    for (;;) {
        std::function<void()> f;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->items.empty(); });
            if (s->items.empty()) return;
            f = std::move(s->items.front());
            s->items.pop_front();
        }
        const int pause = g_max_pause_us.load();
        if (pause > 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % (unsigned)pause));
        f();
        s->completed.fetch_add(1, std::memory_order_release);
        {
            std::lock_guard<std::mutex> g(s->mu);  // pairs with hipStreamSynchronize's wait
        }
        s->cv.notify_all();
    }
}

}  // namespace

// ---- timed condition-variable waits --------------------------------------
// libstdc++ waits on the steady clock with pthread_cond_clockwait, which this
// toolchain's ThreadSanitizer runtime does not intercept: it would not see
// the wait release and retake the mutex, and would report the next lock of
// it as a double lock.  This definition (found before the C library's)
// routes such waits through pthread_cond_timedwait, which it intercepts,
// converting the deadline to the condition's default realtime clock.
extern "C" int pthread_cond_clockwait(pthread_cond_t* cond, pthread_mutex_t* mutex, clockid_t clock,
                                      const struct timespec* abstime) {
    timespec now_c, now_rt;
    clock_gettime(clock, &now_c);
    clock_gettime(CLOCK_REALTIME, &now_rt);
    long long ns = (long long)(abstime->tv_sec - now_c.tv_sec) * 1000000000LL + (abstime->tv_nsec - now_c.tv_nsec);
    if (ns < 0) ns = 0;
    long long t = (long long)now_rt.tv_nsec + ns;
    timespec until;
    until.tv_sec = now_rt.tv_sec + (time_t)(t / 1000000000LL);
    until.tv_nsec = (long)(t % 1000000000LL);
    return pthread_cond_timedwait(cond, mutex, &until);
}

// ---- HIP stand-ins -------------------------------------------------------
hipError_t hipGetDevice(int* d) {
    *d = t_device;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) {
    t_device = d;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* out, unsigned) {
    StubStream* s = new StubStream;
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->completed.load(std::memory_order_acquire) == s->submitted; });
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    hipStreamSynchronize(s);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
    delete s;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    *e = new StubEvent;
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::mutex> g(s->mu);
    e->stream = s;
    e->seq = s->submitted;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    if (!e->stream) return hipSuccess;
    return e->stream->completed.load(std::memory_order_acquire) >= e->seq ? hipSuccess : hipErrorNotReady;
}
const char* hipGetErrorString(hipError_t) { return "simulated device error"; }

// ---- library stand-ins ---------------------------------------------------
namespace rtv {

int set_last_error(int status, const char* msg) {
    t_error = msg;
    return status;
}
int storage_layout_kind(int storage, int layout) {
    return storage >= 0 && storage <= 6 && layout >= 0 && layout <= 4 ? storage * 8 + layout : -1;
}
int volume_kind(const rt_volume* v) { return v ? v->kind : -1; }
bool unit_range(const float* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!(v[i] >= 0.0f && v[i] <= 1.0f)) return false;
    return true;
}
int check_request(const rt_volume* vol, int K, double vmin, double vmax, const void* camera, int W, int H, double,
                  double, const float*, const float*, int ray_function, float, float, double, int* kind) {
    if (!vol || !camera) return set_last_error(RT_ERR_INVALID_ARG, "NULL volume or camera");
    if (K < 2 || K > kMaxK) return set_last_error(RT_ERR_INVALID_ARG, "K out of range");
    if (!(vmax > vmin)) return set_last_error(RT_ERR_INVALID_ARG, "need vmin < vmax");
    if (W < 1 || H < 1 || W > 32768 || H > 32768) return set_last_error(RT_ERR_INVALID_ARG, "bad image size");
    if (ray_function < 0 || ray_function > 5) return set_last_error(RT_ERR_INVALID_ARG, "bad ray function");
    *kind = vol->kind;
    return RT_OK;
}

}  // namespace rtv

extern "C" {

const char* rt_last_error(void) { return t_error.c_str(); }

rt_status rt_tf_bytes(int K, size_t* bytes) {
    *bytes = (size_t)K * 16;
    return RT_OK;
}

rt_status rt_batch_workspace_bytes(int max_jobs, size_t* bytes) {
    *bytes = 256 + (size_t)max_jobs * 64;
    return RT_OK;
}

rt_status rt_set_transfer_function(rt_tf** tf, const float* rgba, int K, double, double, void* dev_buf, size_t,
                                   void* stream) {
    if (!tf || !rgba || K < 2 || K > rtv::kMaxK) return RT_ERR_INVALID_ARG;
    if (*tf && K > (*tf)->cap) return RT_ERR_OUT_OF_MEMORY;  // as the library: K may change within the buffers
    if (!*tf) *tf = new rt_tf{K, K, static_cast<float*>(dev_buf)};
    (*tf)->K = K;
    // staged synchronously, as the library stages the caller's table before the copy
    std::vector<float> staged(rgba, rgba + 4 * (size_t)K);
    float* dst = (*tf)->dev;
    enqueue(static_cast<StubStream*>(stream), [dst, staged] { std::memcpy(dst, staged.data(), staged.size() * 4); });
    return RT_OK;
}

rt_status rt_destroy_tf(rt_tf* tf) {
    delete tf;
    return RT_OK;
}

rt_status rt_batch_plan_create(int max_jobs, int storage, int layout, void*, size_t, const rt_render_opts* opts,
                               rt_batch_plan** out) {
    if (opts && (opts->batch_form < 0 || opts->batch_form > 2)) return RT_ERR_INVALID_ARG;
    *out = new rt_batch_plan{max_jobs, rtv::storage_layout_kind(storage, layout)};
    return RT_OK;
}

rt_status rt_batch_plan_launch(rt_batch_plan* p, const rt_render_job* jobs, int n, unsigned long long* counter,
                               void* stream) {
    if (!p || !jobs || n < 1 || n > p->max_jobs) return RT_ERR_INVALID_ARG;
    struct J {
        float* out;
        int W, H;
        const float* table;
        float eye0;
    };
    std::vector<J> js;
    long px = 0;
    for (int i = 0; i < n; ++i) px += (long)jobs[i].width * jobs[i].height;
    if (n > 1) {
        long seen = g_max_multi_batch_pixels.load();
        while (px > seen && !g_max_multi_batch_pixels.compare_exchange_weak(seen, px)) {
        }
    }
    for (int i = 0; i < n; ++i) {
        if (jobs[i].volume->kind != p->kind) return RT_ERR_INVALID_ARG;
        js.push_back({jobs[i].out_dev, jobs[i].width, jobs[i].height, jobs[i].tf->dev, (float)jobs[i].camera.eye[0]});
    }
    enqueue(static_cast<StubStream*>(stream), [js, counter] {
        for (const J& j : js) {
            const float a = j.table[3];  // the slot the server uploaded on this stream
            for (long k = 0; k < (long)j.W * j.H; ++k) {
                j.out[4 * k + 0] = (float)j.W;
                j.out[4 * k + 1] = (float)j.H;
                j.out[4 * k + 2] = a;
                j.out[4 * k + 3] = j.eye0;
            }
            if (counter) __atomic_fetch_add(counter, (unsigned long long)j.W * j.H, __ATOMIC_RELAXED);
            g_jobs_rendered.fetch_add(1);
        }
    });
    return RT_OK;
}

// Small, so that the server's per-batch pixel cap (16 times this) binds in
// the driver's scenarios.
long long rt_batch_latency_pixels(void) { return 40; }

rt_status rt_batch_plan_destroy(rt_batch_plan* p) {
    delete p;
    return RT_OK;
}

}  // extern "C"
