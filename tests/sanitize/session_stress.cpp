// Host-side stress driver of the serving loop for sanitizer builds (ThreadSanitizer,
// AddressSanitizer): fake sessions only (no device work), through the C ABI.
//
// Exercises: many client threads submitting, waiting and polling at once; cancellation of queued
// requests; requests split into parts; admission under a small budget (with bypass); injected
// launch failures; the watchdog; the open-loop replay harness; close while launches run; argument
// errors of every session call.  Exits non-zero on any unexpected status.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "frg_testing.h"

static std::atomic<int> g_bad{0};

#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            g_bad++;                                                             \
        }                                                                        \
    } while (0)

static frg_integral_desc two_point(int n_q, int n_x) {
    frg_integral_desc d{};
    d.family = FRG_FAMILY_TWO_POINT;
    d.d = 4;
    d.n_q = n_q;
    d.n_x = n_x;
    d.q_max = 10.0;
    d.k = 1.0;
    return d;
}

static frg_integral_desc three_point(int n_q, int n_x, int n_phi) {
    frg_integral_desc d{};
    d.family = FRG_FAMILY_THREE_POINT;
    d.d = 4;
    d.n_q = n_q;
    d.n_x = n_x;
    d.n_phi = n_phi;
    d.q_max = 10.0;
    d.k = 1.0;
    return d;
}

struct Req {
    std::vector<double> ext, out;
    frg_batch b{};
    Req(int n, int ext_per_point) : ext((size_t)n * ext_per_point), out((size_t)n) {
        for (size_t i = 0; i < ext.size(); ++i) ext[i] = 0.01 + 1e-3 * (double)i;
        b.n_ext = n;
        b.ext = ext.data();
        b.m2_scalar = 0.5;
        b.Z = frg_log_table{nullptr, 0, 1e-3, 1e3};
        b.out = out.data();
    }
};

static void clients(frg_session *s, int n_threads, int per_thread) {
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t)
        th.emplace_back([=] {
            std::mt19937 rng(1234 + t);
            for (int k = 0; k < per_thread; ++k) {
                const int n = 16 + (int)(rng() % 300);
                Req r(n, 1);
                const frg_integral_desc d = two_point(8 + (int)(rng() % 24), 4 + (int)(rng() % 12));
                uint64_t ticket = 0;
                frg_status st = frg_session_submit(s, &d, &r.b, -1, &ticket);
                EXPECT(st == FRG_OK);
                if (st != FRG_OK) continue;
                if (k % 7 == 3) {
                    // cancel if still queued; either way the ticket ends
                    st = frg_session_cancel(s, ticket);
                    EXPECT(st == FRG_OK || st == FRG_E_NOTREADY);
                    st = frg_session_wait(s, ticket, -1);
                    EXPECT(st == FRG_OK || st == FRG_E_CANCELLED);
                } else if (k % 5 == 1) {
                    int done = 0;
                    do {
                        st = frg_session_poll(s, ticket, &done);
                        EXPECT(st == FRG_OK);
                        std::this_thread::yield();
                    } while (st == FRG_OK && !done);
                } else {
                    EXPECT(frg_session_wait(s, ticket, -1) == FRG_OK);
                }
            }
        });
    for (auto &x : th) x.join();
}

int main() {
    // 1. many clients on a fake session with room for a few requests at a time
    {
        frg_session_config cfg{4, 256 << 10, 5, 0};
        frg_session *s = nullptr;
        EXPECT(frg_session_open_fake(&cfg, 20.0, 50.0, &s) == FRG_OK);
        clients(s, 16, 60);
        frg_stats st{};
        EXPECT(frg_session_stats(s, &st) == FRG_OK);
        EXPECT(st.failed == 0 && st.tickets_held == 0);
        EXPECT(st.completed + st.cancelled == 16 * 60);
        EXPECT(frg_session_close(s) == FRG_OK);
    }
    // 2. split requests next to small ones, injected failures, then close while busy
    {
        frg_session_config cfg{3, 1 << 30, 5, 0};
        frg_session *s = nullptr;
        EXPECT(frg_session_open_fake(&cfg, 0.05, 20.0, &s) == FRG_OK);
        Req big(4096, 2);
        const frg_integral_desc d3 = three_point(128, 64, 16);  // 5.4e8 nodes: parts
        uint64_t tb = 0;
        EXPECT(frg_session_submit(s, &d3, &big.b, -1, &tb) == FRG_OK);
        EXPECT(frg_session_fake_fail_launches(s, 2) == FRG_OK);
        std::vector<Req> small;
        for (int i = 0; i < 40; ++i) small.emplace_back(64, 1);
        std::vector<uint64_t> ts(small.size());
        const frg_integral_desc d2 = two_point(16, 8);
        for (size_t i = 0; i < small.size(); ++i)
            EXPECT(frg_session_submit(s, &d2, &small[i].b, -1, &ts[i]) == FRG_OK);
        int failed = 0;
        for (uint64_t t : ts) {
            const frg_status st = frg_session_wait(s, t, -1);
            EXPECT(st == FRG_OK || st == FRG_E_DEVICE);
            failed += st == FRG_E_DEVICE;
        }
        const frg_status sb = frg_session_wait(s, tb, -1);
        EXPECT(sb == FRG_OK || sb == FRG_E_DEVICE);
        failed += sb == FRG_E_DEVICE;
        EXPECT(failed >= 1);
        // more work, then close with it in flight
        for (size_t i = 0; i < small.size(); ++i)
            EXPECT(frg_session_submit(s, &d2, &small[i].b, -1, &ts[i]) == FRG_OK);
        EXPECT(frg_session_close(s) == FRG_OK);
    }
    // 3. the watchdog fails a launch that outlives it
    {
        frg_session_config cfg{1, 1 << 20, 5, 20};
        frg_session *s = nullptr;
        EXPECT(frg_session_open_fake(&cfg, 0.0, 100000.0, &s) == FRG_OK);
        Req r(32, 1);
        const frg_integral_desc d = two_point(8, 4);
        uint64_t t = 0;
        EXPECT(frg_session_submit(s, &d, &r.b, -1, &t) == FRG_OK);
        EXPECT(frg_session_wait(s, t, -1) == FRG_E_TIMEOUT);
        EXPECT(frg_session_close(s) == FRG_OK);
    }
    // 4. the open-loop replay harness on a fake session
    {
        frg_session_config cfg{4, 1 << 30, 5, 0};
        frg_session *s = nullptr;
        EXPECT(frg_session_open_fake(&cfg, 1.0, 30.0, &s) == FRG_OK);
        std::vector<double> ext(512), m2(256, 0.5);
        for (size_t i = 0; i < ext.size(); ++i) ext[i] = 0.01 + 1e-2 * (double)i;
        frg_replay_kind kinds[2] = {};
        kinds[0].desc = two_point(16, 8);
        kinds[0].n_ext = 256;
        kinds[1].desc = three_point(16, 8, 4);
        kinds[1].n_ext = 128;
        for (auto &k : kinds) {
            k.ext = ext.data();
            k.m2 = m2.data();
            k.table_id = -1;
            k.x_min = 1e-3;
            k.x_max = 1e3;
        }
        std::vector<frg_replay_arrival> arr(600);
        for (size_t i = 0; i < arr.size(); ++i) arr[i] = frg_replay_arrival{20.0 * (double)i, (int)(i % 2)};
        std::vector<frg_replay_result> res(arr.size());
        double wall = 0.0;
        EXPECT(frg_serving_replay(nullptr, s, 0, 2, kinds, (int)arr.size(), arr.data(), 16,
                                  res.data(), &wall) == FRG_OK);
        for (const auto &x : res) EXPECT(x.status == FRG_OK && x.latency_us >= 0.0);
        EXPECT(frg_session_close(s) == FRG_OK);
    }
    // 5. argument errors, no session state touched
    {
        uint64_t t = 0;
        int done = 0;
        frg_stats st{};
        EXPECT(frg_session_submit(nullptr, nullptr, nullptr, -1, &t) == FRG_E_INVAL);
        EXPECT(frg_session_poll(nullptr, 1, &done) == FRG_E_INVAL);
        EXPECT(frg_session_wait(nullptr, 1, 0) == FRG_E_INVAL);
        EXPECT(frg_session_cancel(nullptr, 1) == FRG_E_INVAL);
        EXPECT(frg_session_stats(nullptr, &st) == FRG_E_INVAL);
        EXPECT(frg_session_close(nullptr) == FRG_OK);
        frg_session_config bad{0, 1 << 20, 5, 0};
        frg_session *s = nullptr;
        EXPECT(frg_session_open_fake(&bad, 1.0, 1.0, &s) == FRG_E_INVAL);
        EXPECT(frg_integrate_batch(nullptr, nullptr, nullptr, nullptr) == FRG_E_INVAL);
        EXPECT(frg_serving_replay(nullptr, nullptr, 0, 0, nullptr, 0, nullptr, 1, nullptr, nullptr) == FRG_E_INVAL);
    }
    if (g_bad) {
        std::fprintf(stderr, "%d expectations failed\n", g_bad.load());
        return 1;
    }
    std::printf("session stress: ok\n");
    return 0;
}
