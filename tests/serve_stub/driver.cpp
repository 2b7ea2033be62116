// Concurrency scenarios for the serving runtime on the simulated device
// (stub_device.cpp), run under ThreadSanitizer by tests/test_serve_tsan.py.
// Test infrastructure only.  Exit status 0 when every check holds; each
// failed check prints one line.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "rt.h"
#include "rt_serve.h"

struct rt_volume {
    int kind;
};
extern std::atomic<long> g_jobs_rendered;
extern std::atomic<int> g_max_pause_us;
extern std::atomic<long> g_max_multi_batch_pixels;
int hipSetDevice(int);
int hipGetDevice(int*);

namespace {

std::atomic<int> g_failures{0};
std::mutex g_print;

#define CHECK(cond, ...)                                                 \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::lock_guard<std::mutex> g_(g_print);                     \
            std::fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                           \
            std::fprintf(stderr, "\n");                                  \
            g_failures.fetch_add(1);                                     \
        }                                                                \
    } while (0)

constexpr int kStorage = 6, kLayout = 4;  // any pair the stub knows
rt_volume g_volume{kStorage * 8 + kLayout};
rt_volume g_other{1 * 8 + 0};

size_t r256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Server {
    rt_server* s = nullptr;
    void* arena = nullptr;
    Server(int streams, int max_batch, size_t pool) {
        size_t bytes = 0;
        CHECK(rt_server_arena_bytes(streams, max_batch, pool, &bytes) == RT_OK, "arena bytes");
        arena = std::aligned_alloc(256, r256(bytes));
        rt_render_opts o;
        std::memset(&o, 0, sizeof(o));
        o.skip_empty = 1;
        CHECK(rt_server_create(streams, max_batch, kStorage, kLayout, &o, arena, r256(bytes), pool, &s) == RT_OK,
              "create: %s", rt_last_error());
    }
    void destroy() {
        if (s) rt_server_destroy(s);
        s = nullptr;
    }
    ~Server() {
        destroy();
        std::free(arena);
    }
};

// One request of a client: its table's first alpha and its camera's eye.x
// identify it in the image the stub writes.
struct Mine {
    std::vector<float> table;
    rt_request req;
};

Mine make_request(std::mt19937& rng, int W, int H) {
    Mine m;
    const int K = 2 + (int)(rng() % 63);
    m.table.resize(4 * (size_t)K);
    for (float& v : m.table) v = (float)(rng() % 1000) / 999.0f;
    std::memset(&m.req, 0, sizeof(m.req));
    m.req.volume = &g_volume;
    m.req.tf_entries = K;
    m.req.tf_vmin = 0.0;
    m.req.tf_vmax = 4095.0;
    m.req.camera.eye[0] = (double)(rng() % 100000);
    m.req.camera.eye[1] = 1.0;
    m.req.camera.up[2] = 1.0;
    m.req.camera.perspective = 1;
    m.req.camera.fovy_deg = 30.0;
    m.req.width = W;
    m.req.height = H;
    m.req.step_vox = 0.5;
    m.req.alpha_cutoff = 0.99;
    m.req.tf_rgba = m.table.data();
    return m;
}

void check_image(const rt_request_info& info, const Mine& m, const char* what) {
    CHECK(info.state == RT_REQ_DONE, "%s: state %d", what, info.state);
    if (info.state != RT_REQ_DONE) return;
    CHECK(info.t_submit > 0 && info.t_submit <= info.t_launch && info.t_launch <= info.t_done, "%s: stamps", what);
    CHECK(info.batch_size >= 1, "%s: batch size", what);
    const float* p = info.image_dev;
    const long n = (long)m.req.width * m.req.height;
    for (long k = 0; k < n; ++k) {
        if (p[4 * k] != (float)m.req.width || p[4 * k + 1] != (float)m.req.height || p[4 * k + 2] != m.table[3] ||
            p[4 * k + 3] != (float)m.req.camera.eye[0]) {
            CHECK(false, "%s: pixel %ld of a %dx%d image is not the request's", what, k, m.req.width, m.req.height);
            return;
        }
    }
}

// Several clients submit, peek, wait for and release their own requests at
// once, in bursts, against a pool that holds only part of them; each client
// overwrites its tables as soon as submit returns and checks its images.
void concurrent_clients() {
    const size_t pool = 24 * r256(24 * 24 * 16);
    Server S(3, 8, pool);
    std::vector<std::thread> th;
    for (int c = 0; c < 6; ++c)
        th.emplace_back([&, c] {
            std::mt19937 rng(100 + c);
            hipSetDevice(c % 2);  // the server's calls must not disturb the caller's device
            for (int round = 0; round < 12; ++round) {
                const int burst = 1 + (int)(rng() % 5);
                std::vector<Mine> ms(burst);
                std::vector<std::vector<float>> keep(burst);
                std::vector<uint64_t> ts(burst);
                for (int b = 0; b < burst; ++b) {
                    ms[b] = make_request(rng, 1 + (int)(rng() % 24), 1 + (int)(rng() % 24));
                    ms[b].req.tf_rgba = ms[b].table.data();
                    keep[b] = ms[b].table;
                    CHECK(rt_server_submit(S.s, &ms[b].req, &ts[b]) == RT_OK, "submit: %s", rt_last_error());
                    std::fill(ms[b].table.begin(), ms[b].table.end(), 0.5f);  // the server holds its own copy
                }
                int dev = -1;
                hipGetDevice(&dev);
                CHECK(dev == c % 2, "caller's device changed to %d", dev);
                for (int b = 0; b < burst; ++b) {
                    rt_request_info info;
                    CHECK(rt_server_wait(S.s, ts[b], 0.0, &info) == RT_OK, "peek");
                    CHECK(rt_server_wait(S.s, ts[b], -1.0, &info) == RT_OK, "wait");
                    ms[b].table = keep[b];
                    check_image(info, ms[b], "concurrent client");
                    CHECK(rt_server_release(S.s, ts[b]) == RT_OK, "release");
                    CHECK(rt_server_release(S.s, ts[b]) == RT_ERR_INVALID_ARG, "second release");
                }
            }
        });
    for (auto& t : th) t.join();
    rt_server_stats st;
    CHECK(rt_server_get_stats(S.s, &st) == RT_OK, "stats");
    CHECK(st.completed == st.submitted && st.failed == 0 && st.queued == 0 && st.running == 0,
          "stats: %llu submitted, %llu completed, %llu failed, %d queued, %d running", st.submitted, st.completed,
          st.failed, st.queued, st.running);
    CHECK(st.pool_in_use == 0 && st.pool_peak <= pool, "pool: in use %zu, peak %zu of %zu", st.pool_in_use,
          st.pool_peak, pool);
}

// Image contents per request: the table is copied at submission, so the
// client may overwrite it at once; each image carries its request's values.
void images_are_the_requests() {
    Server S(2, 4, 64 * r256(16 * 16 * 16));
    std::vector<std::thread> th;
    for (int c = 0; c < 4; ++c)
        th.emplace_back([&, c] {
            std::mt19937 rng(500 + c);
            for (int k = 0; k < 40; ++k) {
                Mine m = make_request(rng, 1 + (int)(rng() % 16), 1 + (int)(rng() % 16));
                const std::vector<float> keep = m.table;
                uint64_t t = 0;
                CHECK(rt_server_submit(S.s, &m.req, &t) == RT_OK, "submit");
                std::fill(m.table.begin(), m.table.end(), 0.25f);  // reused at once
                rt_request_info info;
                CHECK(rt_server_wait(S.s, t, -1.0, &info) == RT_OK, "wait");
                m.table = keep;
                check_image(info, m, "image");
                CHECK(rt_server_release(S.s, t) == RT_OK, "release");
            }
        });
    for (auto& t : th) t.join();
}

// A pool of two images: requests wait for memory and leave the queue in
// submission order, whichever thread submitted them.
void first_come_first_served() {
    const size_t img = r256(16 * 16 * 16);
    Server S(2, 4, 2 * img);
    std::mutex mu;
    std::vector<std::pair<uint64_t, double>> launched;
    std::vector<std::thread> th;
    for (int c = 0; c < 4; ++c)
        th.emplace_back([&, c] {
            std::mt19937 rng(900 + c);
            for (int k = 0; k < 25; ++k) {
                Mine m = make_request(rng, 16, 16);
                uint64_t t = 0;
                CHECK(rt_server_submit(S.s, &m.req, &t) == RT_OK, "submit");
                rt_request_info info;
                CHECK(rt_server_wait(S.s, t, -1.0, &info) == RT_OK, "wait");
                check_image(info, m, "fcfs image");
                {
                    std::lock_guard<std::mutex> g(mu);
                    launched.push_back({t, info.t_launch});
                }
                CHECK(rt_server_release(S.s, t) == RT_OK, "release");
            }
        });
    for (auto& t : th) t.join();
    std::sort(launched.begin(), launched.end());
    for (size_t i = 1; i < launched.size(); ++i)
        CHECK(launched[i].second >= launched[i - 1].second, "ticket %llu left the queue before ticket %llu",
              (unsigned long long)launched[i].first, (unsigned long long)launched[i - 1].first);
    rt_server_stats st;
    rt_server_get_stats(S.s, &st);
    CHECK(st.pool_peak <= 2 * img, "pool peak %zu above %zu", st.pool_peak, 2 * img);
}

// Ticket rules and rejections, with other clients running.
void ticket_rules() {
    const size_t img = r256(8 * 8 * 16);
    Server S(1, 2, img);
    std::mt19937 rng(7);
    Mine a = make_request(rng, 8, 8), b = make_request(rng, 8, 8);
    uint64_t ta = 0, tb = 0;
    CHECK(rt_server_submit(S.s, &a.req, &ta) == RT_OK, "submit a");
    CHECK(rt_server_submit(S.s, &b.req, &tb) == RT_OK, "submit b");
    rt_request_info info;
    CHECK(rt_server_wait(S.s, ta, -1.0, &info) == RT_OK && info.state == RT_REQ_DONE, "a done");
    CHECK(rt_server_wait(S.s, tb, 0.01, &info) == RT_OK && info.state == RT_REQ_QUEUED, "b waits for a's memory");
    CHECK(rt_server_release(S.s, tb) == RT_ERR_INVALID_ARG, "release of a queued request");
    CHECK(rt_server_release(S.s, 999999) == RT_ERR_INVALID_ARG, "release of an unknown ticket");
    CHECK(rt_server_wait(S.s, 999999, 0.0, &info) == RT_ERR_INVALID_ARG, "wait on an unknown ticket");
    Mine big = make_request(rng, 64, 64);
    uint64_t t = 0;
    CHECK(rt_server_submit(S.s, &big.req, &t) == RT_ERR_OUT_OF_MEMORY, "image larger than the pool");
    Mine other = make_request(rng, 4, 4);
    other.req.volume = &g_other;
    CHECK(rt_server_submit(S.s, &other.req, &t) == RT_ERR_INVALID_ARG, "volume of another storage type");
    Mine bad = make_request(rng, 4, 4);
    bad.table[5] = 1.5f;
    CHECK(rt_server_submit(S.s, &bad.req, &t) == RT_ERR_INVALID_ARG, "table value above 1");
    CHECK(rt_server_release(S.s, ta) == RT_OK, "release a");
    CHECK(rt_server_wait(S.s, tb, -1.0, &info) == RT_OK, "b");
    check_image(info, b, "b after a's release");
    CHECK(rt_server_release(S.s, tb) == RT_OK, "release b");
}

// Shutdown: queued and running work finishes; a request that can never be
// admitted (unreleased images hold the pool) fails instead of being waited for.
void shutdown_paths() {
    {
        const size_t img = r256(16 * 16 * 16);
        Server S(1, 4, img);
        std::mt19937 rng(11);
        std::vector<Mine> ms;
        std::vector<uint64_t> ts;
        for (int k = 0; k < 3; ++k) {
            ms.push_back(make_request(rng, 16, 16));
            uint64_t t = 0;
            CHECK(rt_server_submit(S.s, &ms.back().req, &t) == RT_OK, "submit");
            ts.push_back(t);
        }
        rt_request_info info;
        CHECK(rt_server_wait(S.s, ts[0], -1.0, &info) == RT_OK && info.state == RT_REQ_DONE, "first done");
        const auto t0 = std::chrono::steady_clock::now();
        S.destroy();
        const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        CHECK(s < 5.0, "destroy took %.1f s", s);
    }
    {
        const long before = g_jobs_rendered.load();
        Server S(2, 2, 64 * r256(12 * 12 * 16));
        std::vector<std::thread> th;
        std::vector<Mine> keep[3];
        for (int c = 0; c < 3; ++c)
            th.emplace_back([&, c] {
                std::mt19937 rng(40 + c);
                for (int k = 0; k < 10; ++k) {
                    keep[c].push_back(make_request(rng, 12, 12));
                    uint64_t t = 0;
                    CHECK(rt_server_submit(S.s, &keep[c].back().req, &t) == RT_OK, "submit");
                }
            });
        for (auto& t : th) t.join();
        S.destroy();  // returns once all 30 have rendered
        CHECK(g_jobs_rendered.load() - before == 30, "%ld of 30 rendered before destroy returned",
              g_jobs_rendered.load() - before);
    }
}

}  // namespace

int main() {
    concurrent_clients();
    images_are_the_requests();
    first_come_first_served();
    ticket_rules();
    g_max_pause_us.store(2000);  // slower batches: more requests queue behind running ones
    shutdown_paths();
    concurrent_clients();
    // batches of several requests stay within the pixel cap (16 x the stub's 40)
    CHECK(g_max_multi_batch_pixels.load() > 0 && g_max_multi_batch_pixels.load() <= 16 * 40,
          "largest multi-request batch: %ld pixels", g_max_multi_batch_pixels.load());
    const int f = g_failures.load();
    std::printf("%s: %d failed checks\n", f ? "FAILED" : "ok", f);
    return f ? 1 : 0;
}
