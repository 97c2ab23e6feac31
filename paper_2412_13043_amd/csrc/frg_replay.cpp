// Open-loop replay of a request arrival trace, for measuring the serving loop against the plain
// per-batch path with one and the same client harness (no interpreter in the timing loop).
//
// Mode 0 (session): the calling thread submits each arrival to the session at its arrival time;
// a pool of waiter threads blocks on the tickets and stamps each completion, so a request's
// latency is completion - arrival time, the result already in its host buffer.
// Mode 1 (plain path): one thread serves the arrivals first-in first-out on one stream, each by
// copying its inputs to the device, one frg_integrate_batch in float64, and copying the result
// back; a request waits until the previous one has finished.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/frg_testing.h"
#include "frg_runtime.hpp"

namespace frg {

static double replay_now_us() {
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// Sleep most of the way to `t_us`, then spin the rest (arrival times to about a microsecond).
static void wait_until(double t_us) {
    for (;;) {
        const double d = t_us - replay_now_us();
        if (d <= 0.0) return;
        if (d > 300.0)
            std::this_thread::sleep_for(std::chrono::microseconds((long long)(d - 200.0)));
    }
}

static bool same_bits(const double *a, const double *b, int n) {
    return std::memcmp(a, b, (size_t)n * sizeof(double)) == 0;
}

// Output buffers of one kind of request: a few reusable ones, more when they are all in use.
struct KindBuffers {
    std::vector<std::vector<double>> out, err;
    std::vector<int> free_list;
    int take(int n) {
        if (free_list.empty()) {
            out.emplace_back((size_t)n);
            err.emplace_back((size_t)n);
            return (int)out.size() - 1;
        }
        const int b = free_list.back();
        free_list.pop_back();
        return b;
    }
};

struct Pending {
    uint64_t ticket;
    int arrival;
    int buf;
};

static frg_status replay_session(frg_session *s, int n_kinds, const frg_replay_kind *kinds,
                                 int n_arr, const frg_replay_arrival *arr, int n_waiters,
                                 frg_replay_result *res, double *wall_us) {
    std::vector<KindBuffers> bufs((size_t)n_kinds);
    std::mutex mu;  // buffers, the pending queue
    std::condition_variable cv;
    std::deque<Pending> pending;
    bool submitted_all = false;
    double t_last = 0.0;
    const double t0 = replay_now_us() + 1000.0;  // the first arrival a millisecond from now

    auto waiter = [&]() {
        for (;;) {
            Pending p;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return !pending.empty() || submitted_all; });
                if (pending.empty()) return;
                p = pending.front();
                pending.pop_front();
            }
            const frg_status st = frg_session_wait(s, p.ticket, -1);
            const double t = replay_now_us();
            const frg_replay_arrival &a = arr[p.arrival];
            const frg_replay_kind &k = kinds[a.kind];
            frg_replay_result &r = res[p.arrival];
            r.latency_us = t - (t0 + a.t_us);
            r.status = st;
            std::lock_guard<std::mutex> lk(mu);
            r.mismatch = (st == FRG_OK && k.expect &&
                          !same_bits(bufs[a.kind].out[p.buf].data(), k.expect, k.n_ext))
                             ? 1
                             : 0;
            bufs[a.kind].free_list.push_back(p.buf);
            t_last = std::max(t_last, t);
        }
    };
    std::vector<std::thread> pool;
    for (int i = 0; i < n_waiters; ++i) pool.emplace_back(waiter);
    frg_status bad = FRG_OK;
    for (int i = 0; i < n_arr; ++i) {
        const frg_replay_arrival &a = arr[i];
        const frg_replay_kind &k = kinds[a.kind];
        int b;
        frg_batch batch{};
        {
            std::lock_guard<std::mutex> lk(mu);
            b = bufs[a.kind].take(k.n_ext);
            batch.out = bufs[a.kind].out[b].data();
            batch.err_out = k.desc.precision ? bufs[a.kind].err[b].data() : nullptr;
        }
        batch.n_ext = k.n_ext;
        batch.ext = k.ext;
        batch.m2 = k.m2;
        batch.Z = frg_log_table{nullptr, 0, k.x_min, k.x_max};
        wait_until(t0 + a.t_us);
        uint64_t ticket = 0;
        const frg_status st = frg_session_submit(s, &k.desc, &batch, k.table_id, &ticket);
        if (st != FRG_OK) {
            res[i].status = st;
            res[i].latency_us = -1.0;
            bad = st;
            std::lock_guard<std::mutex> lk(mu);
            bufs[a.kind].free_list.push_back(b);
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            pending.push_back(Pending{ticket, i, b});
        }
        cv.notify_one();
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        submitted_all = true;
    }
    cv.notify_all();
    for (auto &t : pool) t.join();
    *wall_us = t_last - t0;
    if (bad != FRG_OK) set_error("some submissions failed (status %d)", bad);
    return bad;
}

static frg_status replay_plain(frg_context *ctx, int n_kinds, const frg_replay_kind *kinds,
                               int n_arr, const frg_replay_arrival *arr, frg_replay_result *res,
                               double *wall_us) {
    size_t max_ext = 1, max_n = 1;
    for (int i = 0; i < n_kinds; ++i) {
        max_ext = std::max(max_ext, (size_t)ext_values(kinds[i].desc, kinds[i].n_ext));
        max_n = std::max(max_n, (size_t)kinds[i].n_ext);
    }
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    DeviceBuffer d_ext, d_m2, d_out;
    FRG_HIP_CHECK(d_ext.alloc(max_ext * sizeof(double)));
    FRG_HIP_CHECK(d_m2.alloc(max_n * sizeof(double)));
    FRG_HIP_CHECK(d_out.alloc(max_n * sizeof(double)));
    void *stage = nullptr;
    const size_t stage_bytes = (max_ext + 2 * max_n) * sizeof(double);
    FRG_HIP_CHECK(hipHostMalloc(&stage, stage_bytes, hipHostMallocDefault));
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipHostFree(stage);
        set_error("hipStreamCreateWithFlags failed");
        return FRG_E_DEVICE;
    }
    std::vector<double> out(max_n);
    frg_status bad = FRG_OK;
    const double t0 = replay_now_us() + 1000.0;
    double t_last = t0;
    double *h_ext = (double *)stage, *h_m2 = h_ext + max_ext, *h_out = h_m2 + max_n;
    for (int i = 0; i < n_arr && bad == FRG_OK; ++i) {
        const frg_replay_arrival &a = arr[i];
        const frg_replay_kind &k = kinds[a.kind];
        wait_until(t0 + a.t_us);  // first in, first out: no earlier than the previous one ends
        const size_t ne = (size_t)ext_values(k.desc, k.n_ext);
        if (ne) std::memcpy(h_ext, k.ext, ne * sizeof(double));
        std::memcpy(h_m2, k.m2, (size_t)k.n_ext * sizeof(double));
        frg_integral_desc d = k.desc;
        d.precision = FRG_FP64;  // the plain path is float64
        d.near_pole_tau = 0.0;
        frg_batch b{};
        b.n_ext = k.n_ext;
        b.ext = ne ? (const double *)d_ext.ptr : nullptr;
        b.m2 = (const double *)d_m2.ptr;
        b.Z = frg_log_table{k.Z_dev, k.Z_dev ? k.nZ : 0, k.x_min, k.x_max};
        b.out = (double *)d_out.ptr;
        hipError_t e = hipSuccess;
        if (ne) e = hipMemcpyAsync(d_ext.ptr, h_ext, ne * sizeof(double), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_m2.ptr, h_m2, (size_t)k.n_ext * sizeof(double),
                               hipMemcpyHostToDevice, st);
        frg_status fs = e == hipSuccess ? frg_integrate_batch(ctx, &d, &b, st) : FRG_E_DEVICE;
        if (fs == FRG_OK)
            e = hipMemcpyAsync(h_out, d_out.ptr, (size_t)k.n_ext * sizeof(double),
                               hipMemcpyDeviceToHost, st);
        if (fs == FRG_OK && e == hipSuccess) e = hipStreamSynchronize(st);
        if (fs == FRG_OK && e != hipSuccess) {
            set_error("plain-path replay: %s", hipGetErrorString(e));
            fs = FRG_E_DEVICE;
        }
        if (fs == FRG_OK) std::memcpy(out.data(), h_out, (size_t)k.n_ext * sizeof(double));
        const double t = replay_now_us();
        res[i].latency_us = t - (t0 + a.t_us);
        res[i].status = fs;
        res[i].mismatch = (fs == FRG_OK && k.expect && k.desc.precision == FRG_FP64 &&
                           !same_bits(out.data(), k.expect, k.n_ext))
                              ? 1
                              : 0;
        t_last = t;
        if (fs != FRG_OK) bad = fs;
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    (void)hipHostFree(stage);
    *wall_us = t_last - t0;
    return bad;
}

}  // namespace frg

using namespace frg;

extern "C" frg_status frg_serving_replay(frg_context *ctx, frg_session *s, int mode, int n_kinds,
                                         const frg_replay_kind *kinds, int n_arr,
                                         const frg_replay_arrival *arr, int n_waiters,
                                         frg_replay_result *res, double *wall_us) {
    clear_error();
    if (!kinds || n_kinds < 1 || n_arr < 0 || (n_arr > 0 && (!arr || !res)) || !wall_us ||
        (mode == 0 && (!s || n_waiters < 1 || n_waiters > 1024)) || (mode == 1 && !ctx) ||
        (mode != 0 && mode != 1)) {
        set_error("invalid arguments to frg_serving_replay");
        return FRG_E_INVAL;
    }
    for (int i = 0; i < n_arr; ++i)
        if (arr[i].kind < 0 || arr[i].kind >= n_kinds || !(arr[i].t_us >= 0.0) ||
            (i > 0 && arr[i].t_us < arr[i - 1].t_us)) {
            set_error("arrival %d: kind out of range or times not ascending", i);
            return FRG_E_INVAL;
        }
    for (int i = 0; i < n_arr; ++i) res[i] = frg_replay_result{0.0, FRG_OK, 0};
    if (n_arr == 0) {
        *wall_us = 0.0;
        return FRG_OK;
    }
    return mode == 0 ? replay_session(s, n_kinds, kinds, n_arr, arr, n_waiters, res, wall_us)
                     : replay_plain(ctx, n_kinds, kinds, n_arr, arr, res, wall_us);
}
