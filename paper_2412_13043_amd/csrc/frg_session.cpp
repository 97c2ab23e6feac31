// Serving loop: continuous batching of loop-integral requests from many concurrent clients.
//
// Requests are queued by frg_session_submit.  A scheduler thread admits queued requests in
// arrival order while their device footprint (inputs, outputs, contribution scratch) fits in the
// session's HBM arena, packs every admissible request into one fused persistent launch (the
// multi-request tile consumer) on a free launch slot, and keeps up to max_inflight such launches
// on separate streams, so requests that arrive while others run are admitted as memory and slots
// free up and their work overlaps on the device.  A finished launch's outputs are copied back to
// the clients' host buffers before their tickets complete.  Each result is computed exactly as
// frg_integrate_batch would compute it (results do not depend on batch composition).
//
// Execution goes through an Executor interface: the HIP executor above, and a test double that
// runs no device work and completes tickets after a delay proportional to their node count, used
// by CPU-only tests of admission, cancellation, time-outs and accounting.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "../../include/frg_testing.h"
#include "frg_runtime.hpp"

namespace frg {

static double now_us() {
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING, RQ_DONE, RQ_FAILED, RQ_CANCELLED };

struct SessReq {
    uint64_t ticket = 0;
    frg_integral_desc desc{};
    frg_batch host{};    // host pointers from the client
    int table_id = -1;
    int n_ext_vals = 0;  // doubles in ext
    // device layout inside the request's arena block (byte offsets)
    size_t off_ext = 0, off_m2 = 0, off_z = 0, off_out = 0, off_err = 0, off_contrib = 0;
    size_t in_bytes = 0;   // ext + m2 + Z, contiguous from offset 0
    size_t footprint = 0;  // whole block
    size_t arena_off = 0;
    uint64_t nodes = 0;
    double t_submit = 0.0, t_done = 0.0;
    ReqState state = RQ_QUEUED;
    frg_status status = FRG_OK;
    bool timed_out = false;
};

// First-fit allocator over a contiguous device range, 256-byte granularity, coalescing frees.
class Arena {
   public:
    void init(size_t cap) {
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
        used_ = 0;
    }
    static constexpr size_t npos = (size_t)-1;
    size_t alloc(size_t n) {
        n = align256(std::max<size_t>(n, 256));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                size_t off = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used_ += n;
                return off;
            }
        }
        return npos;
    }
    void release(size_t off, size_t n) {
        n = align256(std::max<size_t>(n, 256));
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }

   private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    DeviceBuffer tables;    // ReqDev[] then TileDev[]
    DeviceBuffer counters;  // zeroed before each launch
    DeviceBuffer work;      // fused-launch tile counter (cleared ahead of each launch)
    void *host = nullptr;   // pinned staging: tables, inputs, outputs
    size_t host_bytes = 0;
    std::vector<SessReq *> reqs;
    std::vector<size_t> host_out;  // staging offset of each request's outputs
    bool busy = false;
    double t_launch = 0.0;
    double fake_ready = 0.0;  // test double: completion time
    ~Slot() {
        if (host) (void)hipHostFree(host);
        if (done) (void)hipEventDestroy(done);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

struct ResidentTable {
    DeviceBuffer buf;
    int n = 0;
    double x_min = 0, x_max = 0;
};



class Executor {
   public:
    virtual ~Executor() = default;
    virtual frg_status setup(frg_session &) = 0;
    virtual frg_status launch(frg_session &, Slot &) = 0;
    virtual int poll(frg_session &, Slot &) = 0;  // 1 done, 0 running, -1 device error
    virtual void finish(frg_session &, Slot &) = 0;
};

}  // namespace frg

struct frg_session {
    frg_context *ctx = nullptr;
    frg_session_config cfg{};
    std::unique_ptr<frg::Executor> exec;
    std::mutex mu;
    std::condition_variable cv;
    std::thread thr;
    bool stop = false;
    std::deque<frg::SessReq *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<frg::SessReq>> reqs;
    uint64_t next_ticket = 1;
    frg::Arena arena;
    frg::DeviceBuffer arena_mem;
    std::vector<std::unique_ptr<frg::Slot>> slots;
    std::vector<std::unique_ptr<frg::ResidentTable>> tables;
    double fake_ns_per_node = 0.0, fake_base_us = 0.0;
    // statistics
    std::vector<double> lat_us;
    uint64_t admitted = 0, rejected = 0, completed = 0, failed = 0, cancelled = 0, nodes_done = 0,
             launches = 0;
    double t_first = 0.0, t_last = 0.0;
    std::string fatal;
};

namespace frg {

// ---------------------------------------------------------------------------------------------
// HIP executor
// ---------------------------------------------------------------------------------------------
class HipExecutor : public Executor {
   public:
    frg_status setup(frg_session &s) override {
        FRG_HIP_CHECK(hipSetDevice(s.ctx->device));
        FRG_HIP_CHECK(s.arena_mem.alloc(s.arena.capacity()));
        for (auto &sl : s.slots) {
            FRG_HIP_CHECK(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
            FRG_HIP_CHECK(hipEventCreateWithFlags(&sl->done, hipEventDisableTiming));
            FRG_HIP_CHECK(sl->work.alloc(2 * sizeof(unsigned)));
            FRG_HIP_CHECK(launch_fill_zero_u32((unsigned *)sl->work.ptr, 2, sl->stream));
            FRG_HIP_CHECK(hipStreamSynchronize(sl->stream));
        }
        return FRG_OK;
    }

    frg_status launch(frg_session &s, Slot &sl) override {
        frg_context *ctx = s.ctx;
        std::lock_guard<std::mutex> lk(ctx->mu);
        FRG_HIP_CHECK(hipSetDevice(ctx->device));
        char *base = (char *)s.arena_mem.ptr;
        std::vector<ReqDev> rd;
        double total = 0.0;
        for (SessReq *r : sl.reqs) total += (double)r->nodes;
        const int target_total = 32 * ctx->num_cus;
        long long ctr = 0;
        for (SessReq *r : sl.reqs) {
            frg_batch b = r->host;
            char *blk = base + r->arena_off;
            b.ext = is_vertex(r->desc.family) ? (const double *)(blk + r->off_ext) : nullptr;
            b.m2 = r->host.m2 ? (const double *)(blk + r->off_m2) : nullptr;
            b.out = (double *)(blk + r->off_out);
            b.err_out = r->host.err_out ? (double *)(blk + r->off_err) : nullptr;
            if (r->table_id >= 0) {
                const ResidentTable &t = *s.tables[r->table_id];
                b.Z = frg_log_table{(const double *)t.buf.ptr, t.n, t.x_min, t.x_max};
            } else if (r->host.Z.values) {
                b.Z.values = (const double *)(blk + r->off_z);
            }
            int target = std::max(1, (int)std::lround(target_total * (double)r->nodes / total));
            // session launches run no finalize pass: single-chunk shapes only
            TileShape shape = choose_shape(ctx, r->desc, b.n_ext, target, ShapeUse::kNoChunks);
            ReqDev q;
            frg_status st = make_request(ctx, r->desc, b, shape, 1, 0.0, 1.0, &q);
            if (st != FRG_OK) return st;
            q.contrib_base = (long long)((r->arena_off + r->off_contrib) / sizeof(double));
            q.ctr_base = ctr;
            ctr += counter_count(q);
            rd.push_back(q);
        }
        int lds = 0;
        std::vector<TileDev> tiles = make_tiles(rd, &lds);
        // pinned staging: tables | inputs of each request | outputs of each request
        size_t tb = align256(rd.size() * sizeof(ReqDev)) + align256(tiles.size() * sizeof(TileDev));
        size_t need = tb;
        for (SessReq *r : sl.reqs) need += align256(r->in_bytes);
        size_t out_start = need;
        for (SessReq *r : sl.reqs) need += align256((r->host.err_out ? 2 : 1) * r->host.n_ext * 8);
        if (sl.host_bytes < need) {
            if (sl.host) FRG_HIP_CHECK(hipHostFree(sl.host));
            sl.host = nullptr;
            sl.host_bytes = 0;
            size_t want = need + need / 2 + 65536;
            FRG_HIP_CHECK(hipHostMalloc(&sl.host, want, hipHostMallocDefault));
            sl.host_bytes = want;
        }
        if (sl.tables.bytes < tb) {
            FRG_HIP_CHECK(hipStreamSynchronize(sl.stream));
            if (sl.tables.ptr) FRG_HIP_CHECK(hipFree(sl.tables.ptr));
            sl.tables.ptr = nullptr;
            sl.tables.bytes = 0;
            FRG_HIP_CHECK(sl.tables.alloc(tb + tb / 2 + 4096));
        }
        size_t nctr = std::max<long long>(ctr, 1);
        if (sl.counters.bytes < nctr * sizeof(unsigned)) {
            FRG_HIP_CHECK(hipStreamSynchronize(sl.stream));
            if (sl.counters.ptr) FRG_HIP_CHECK(hipFree(sl.counters.ptr));
            sl.counters.ptr = nullptr;
            sl.counters.bytes = 0;
            FRG_HIP_CHECK(sl.counters.alloc(nctr * sizeof(unsigned) * 2));
        }
        char *h = (char *)sl.host;
        std::memcpy(h, rd.data(), rd.size() * sizeof(ReqDev));
        size_t tiles_off = align256(rd.size() * sizeof(ReqDev));
        std::memcpy(h + tiles_off, tiles.data(), tiles.size() * sizeof(TileDev));
        FRG_HIP_CHECK(hipMemcpyAsync(sl.tables.ptr, h, tb, hipMemcpyHostToDevice, sl.stream));
        size_t pos = tb;
        for (SessReq *r : sl.reqs) {
            char *dst = h + pos;
            const int n = r->host.n_ext;
            if (is_vertex(r->desc.family))
                std::memcpy(dst + r->off_ext, r->host.ext, (size_t)r->n_ext_vals * 8);
            if (r->host.m2) std::memcpy(dst + r->off_m2, r->host.m2, (size_t)n * 8);
            if (r->table_id < 0 && r->host.Z.values && is_vertex(r->desc.family))
                std::memcpy(dst + r->off_z, r->host.Z.values, (size_t)r->host.Z.n * 8);
            if (r->in_bytes)
                FRG_HIP_CHECK(hipMemcpyAsync(base + r->arena_off, dst, r->in_bytes,
                                             hipMemcpyHostToDevice, sl.stream));
            pos += align256(r->in_bytes);
        }
        FRG_HIP_CHECK(launch_fill_zero_u32((unsigned *)sl.counters.ptr, nctr, sl.stream));
        const ReqDev *reqs_dev = (const ReqDev *)sl.tables.ptr;
        const TileDev *tiles_dev = (const TileDev *)((char *)sl.tables.ptr + tiles_off);
        int fam, prec, reg, der;
        common_kind(rd, &fam, &prec, &reg, &der);
        const int grid = multi_grid((int)tiles.size(), fam, prec, reg, der, lds, ctx->num_cus);
        FRG_HIP_CHECK(launch_multi(reqs_dev, fam, prec, reg, der, tiles_dev, (int)tiles.size(),
                                   grid, lds, (double *)base, (unsigned *)sl.counters.ptr,
                                   (unsigned *)sl.work.ptr, sl.stream));
        sl.host_out.clear();
        pos = out_start;
        for (SessReq *r : sl.reqs) {
            const size_t n = (size_t)r->host.n_ext;
            sl.host_out.push_back(pos);
            FRG_HIP_CHECK(hipMemcpyAsync(h + pos, base + r->arena_off + r->off_out, n * 8,
                                         hipMemcpyDeviceToHost, sl.stream));
            if (r->host.err_out)
                FRG_HIP_CHECK(hipMemcpyAsync(h + pos + n * 8, base + r->arena_off + r->off_err,
                                             n * 8, hipMemcpyDeviceToHost, sl.stream));
            pos += align256((r->host.err_out ? 2 : 1) * n * 8);
        }
        FRG_HIP_CHECK(hipEventRecord(sl.done, sl.stream));
        return FRG_OK;
    }

    int poll(frg_session &, Slot &sl) override {
        hipError_t e = hipEventQuery(sl.done);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        set_error("session launch failed: %s", hipGetErrorString(e));
        return -1;
    }

    void finish(frg_session &, Slot &sl) override {
        const char *h = (const char *)sl.host;
        for (size_t i = 0; i < sl.reqs.size(); ++i) {
            SessReq *r = sl.reqs[i];
            if (r->timed_out) continue;
            const size_t n = (size_t)r->host.n_ext;
            std::memcpy(r->host.out, h + sl.host_out[i], n * 8);
            if (r->host.err_out) std::memcpy(r->host.err_out, h + sl.host_out[i] + n * 8, n * 8);
        }
    }
};

// Test double: no device work; a launch completes after base + ns_per_node * nodes.
class FakeExecutor : public Executor {
   public:
    frg_status setup(frg_session &) override { return FRG_OK; }
    frg_status launch(frg_session &s, Slot &sl) override {
        double nodes = 0.0;
        for (SessReq *r : sl.reqs) nodes += (double)r->nodes;
        sl.fake_ready = now_us() + s.fake_base_us + s.fake_ns_per_node * nodes * 1e-3;
        return FRG_OK;
    }
    int poll(frg_session &, Slot &sl) override { return now_us() >= sl.fake_ready ? 1 : 0; }
    void finish(frg_session &, Slot &) override {}
};

// ---------------------------------------------------------------------------------------------
// Scheduler
// ---------------------------------------------------------------------------------------------
static void complete_slot(frg_session &s, Slot &sl, bool ok) {
    double t = now_us();
    if (ok) s.exec->finish(s, sl);
    for (SessReq *r : sl.reqs) {
        s.arena.release(r->arena_off, r->footprint);
        if (r->timed_out) continue;  // already failed by the watchdog
        r->t_done = t;
        if (ok) {
            r->state = RQ_DONE;
            r->status = FRG_OK;
            s.completed++;
            s.nodes_done += r->nodes;
            s.lat_us.push_back(t - r->t_submit);
            s.t_last = t;
        } else {
            r->state = RQ_FAILED;
            r->status = FRG_E_DEVICE;
            s.failed++;
        }
    }
    sl.reqs.clear();
    sl.busy = false;
}

static bool admit_and_launch(frg_session &s) {
    Slot *free_slot = nullptr;
    for (auto &sl : s.slots)
        if (!sl->busy) {
            free_slot = sl.get();
            break;
        }
    if (!free_slot || s.queue.empty()) return false;
    // Arrival order; stop at the first request that does not fit (no overtaking).  A launch
    // completes as a whole, so it is capped at about half a millisecond of the chip: small
    // requests are not held back by a large one launched with them, and a request above the
    // cap runs alone in its slot while the other slots keep serving the rest of the queue.
    const size_t max_reqs = 512;
    const double max_nodes = 2.5e8;
    double nodes = 0.0;
    std::vector<SessReq *> batch;
    while (!s.queue.empty() && batch.size() < max_reqs) {
        SessReq *r = s.queue.front();
        if (!batch.empty() && nodes + (double)r->nodes > max_nodes) break;
        size_t off = s.arena.alloc(r->footprint);
        if (off == Arena::npos) break;
        r->arena_off = off;
        r->state = RQ_RUNNING;
        s.queue.pop_front();
        batch.push_back(r);
        nodes += (double)r->nodes;
    }
    if (batch.empty()) return false;
    free_slot->reqs = batch;
    free_slot->busy = true;
    free_slot->t_launch = now_us();
    s.admitted += batch.size();
    s.launches++;
    frg_status st = s.exec->launch(s, *free_slot);
    if (st != FRG_OK) {
        s.fatal = frg_last_error();
        complete_slot(s, *free_slot, false);
    }
    return true;
}

static void scheduler(frg_session *sp) {
    frg_session &s = *sp;
    if (s.ctx) (void)hipSetDevice(s.ctx->device);
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
        bool progress = false;
        bool busy = false;
        for (auto &sl : s.slots) {
            if (!sl->busy) continue;
            int p = s.exec->poll(s, *sl);
            if (p != 0) {
                complete_slot(s, *sl, p > 0);
                progress = true;
                continue;
            }
            busy = true;
            if (s.cfg.watchdog_ms > 0 && now_us() - sl->t_launch > 1e3 * s.cfg.watchdog_ms) {
                for (SessReq *r : sl->reqs)
                    if (!r->timed_out) {
                        r->timed_out = true;
                        r->state = RQ_FAILED;
                        r->status = FRG_E_TIMEOUT;
                        r->t_done = now_us();
                        s.failed++;
                        progress = true;
                    }
            }
        }
        while (!s.stop && admit_and_launch(s)) progress = true;
        for (auto &sl : s.slots) busy = busy || sl->busy;
        if (progress) s.cv.notify_all();
        if (s.stop && !busy) break;
        if (!progress) {
            if (busy || !s.queue.empty())
                s.cv.wait_for(lk, std::chrono::microseconds(std::max(1, s.cfg.poll_us)));
            else
                s.cv.wait(lk);
        }
    }
    // queued tickets left at close are cancelled
    for (SessReq *r : s.queue) {
        r->state = RQ_CANCELLED;
        r->status = FRG_E_CANCELLED;
        s.cancelled++;
    }
    s.queue.clear();
    s.cv.notify_all();
}

static size_t request_layout(SessReq &r) {
    const frg_integral_desc &d = r.desc;
    const int n = r.host.n_ext;
    size_t off = 0;
    r.n_ext_vals = (int)ext_values(d.family, n);
    r.off_ext = off;
    off += (size_t)r.n_ext_vals * 8;
    r.off_m2 = off;
    if (r.host.m2) off += (size_t)n * 8;
    r.off_z = off;
    if (r.table_id < 0 && r.host.Z.values && is_vertex(d.family)) off += (size_t)r.host.Z.n * 8;
    r.in_bytes = off;
    off = align256(off);
    r.off_out = off;
    off += align256((size_t)n * 8);
    r.off_err = off;
    if (r.host.err_out) off += align256((size_t)n * 8);
    r.off_contrib = off;
    // contributions of radially chunked requests (n_q n_f radial nodes at finite temperature)
    if (is_vertex(d.family)) off += align256((size_t)plan_desc(d).n_q * n * 8);
    return align256(off);
}

static frg_status open_session(frg_context *ctx, const frg_session_config *cfg, bool fake,
                               double ns_per_node, double base_us, frg_session **out) {
    if (!cfg || !out || (!fake && !ctx)) {
        set_error("invalid arguments to frg_session_open");
        return FRG_E_INVAL;
    }
    if (cfg->max_inflight < 1 || cfg->max_inflight > 16 || cfg->poll_us < 0 ||
        cfg->watchdog_ms < 0) {
        set_error("session config needs 1 <= max_inflight <= 16, poll_us >= 0, watchdog_ms >= 0");
        return FRG_E_INVAL;
    }
    auto s = std::make_unique<frg_session>();
    s->ctx = ctx;
    s->cfg = *cfg;
    if (s->cfg.poll_us == 0) s->cfg.poll_us = 20;
    size_t budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (ctx ? ctx->hbm_budget : 0);
    if (budget < 4096) {
        set_error("session HBM budget must be at least 4096 bytes");
        return FRG_E_INVAL;
    }
    s->arena.init(budget & ~(size_t)255);
    for (int i = 0; i < cfg->max_inflight; ++i) s->slots.push_back(std::make_unique<Slot>());
    s->fake_ns_per_node = ns_per_node;
    s->fake_base_us = base_us;
    if (fake)
        s->exec = std::make_unique<FakeExecutor>();
    else
        s->exec = std::make_unique<HipExecutor>();
    frg_status st = s->exec->setup(*s);
    if (st != FRG_OK) return st;
    frg_session *raw = s.get();
    s->thr = std::thread(scheduler, raw);
    *out = s.release();
    return FRG_OK;
}

}  // namespace frg

using namespace frg;

extern "C" {

frg_status frg_session_open(frg_context *ctx, const frg_session_config *cfg, frg_session **out) {
    clear_error();
    return open_session(ctx, cfg, false, 0.0, 0.0, out);
}

frg_status frg_session_open_fake(const frg_session_config *cfg, double ns_per_node,
                                 double base_us, frg_session **out) {
    clear_error();
    if (!(ns_per_node >= 0.0) || !(base_us >= 0.0)) {
        set_error("fake executor needs ns_per_node >= 0 and base_us >= 0");
        return FRG_E_INVAL;
    }
    return open_session(nullptr, cfg, true, ns_per_node, base_us, out);
}

frg_status frg_session_register_table(frg_session *s, const double *Z_host, int n, double x_min,
                                      double x_max, int *table_id) {
    clear_error();
    if (!s || !Z_host || !table_id || n < 2 || n > FRG_MAX_TABLE || !(x_min > 0.0) ||
        !(x_max > x_min)) {
        set_error("invalid dressing table");
        return FRG_E_INVAL;
    }
    auto t = std::make_unique<ResidentTable>();
    t->n = n;
    t->x_min = x_min;
    t->x_max = x_max;
    if (s->ctx) {
        FRG_HIP_CHECK(hipSetDevice(s->ctx->device));
        FRG_HIP_CHECK(t->buf.alloc((size_t)n * sizeof(double)));
        FRG_HIP_CHECK(hipMemcpy(t->buf.ptr, Z_host, (size_t)n * sizeof(double),
                                hipMemcpyHostToDevice));
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->tables.push_back(std::move(t));
    *table_id = (int)s->tables.size() - 1;
    return FRG_OK;
}

frg_status frg_session_submit(frg_session *s, const frg_integral_desc *desc,
                              const frg_batch *batch_host, int table_id, uint64_t *ticket) {
    clear_error();
    if (!s || !ticket) {
        set_error("null session or ticket");
        return FRG_E_INVAL;
    }
    frg_status st = validate(desc, batch_host, false);
    if (st != FRG_OK) return st;
    if (batch_host->dout_dm2) {
        set_error("sessions do not return the mass derivative (dout_dm2 must be NULL)");
        return FRG_E_UNSUPPORTED;
    }
    if (batch_host->dout_dz) {
        set_error("sessions do not return dressing derivatives (dout_dz must be NULL)");
        return FRG_E_UNSUPPORTED;
    }
    auto r = std::make_unique<SessReq>();
    r->desc = *desc;
    r->host = *batch_host;
    r->table_id = table_id;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (table_id >= (int)s->tables.size() || table_id < -1) {
            set_error("unknown table id %d", table_id);
            return FRG_E_INVAL;
        }
        if (s->stop) {
            set_error("session is closing");
            return FRG_E_CANCELLED;
        }
    }
    const frg_integral_desc &d = *desc;
    r->nodes = (uint64_t)((double)batch_host->n_ext * nodes_per_point(d));
    r->footprint = request_layout(*r);
    r->t_submit = now_us();
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->footprint > s->arena.capacity()) {
        s->rejected++;
        set_error("request needs %zu device bytes, more than the session budget %zu",
                  r->footprint, s->arena.capacity());
        return FRG_E_NOMEM;
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    if (s->t_first == 0.0) s->t_first = r->t_submit;
    if (batch_host->n_ext == 0) {
        r->state = RQ_DONE;
        r->t_done = r->t_submit;
        s->completed++;
    } else {
        s->queue.push_back(r.get());
    }
    s->reqs.emplace(r->ticket, std::move(r));
    s->cv.notify_all();
    return FRG_OK;
}

frg_status frg_session_poll(frg_session *s, uint64_t ticket, int *done) {
    clear_error();
    if (!s || !done) {
        set_error("null argument");
        return FRG_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return FRG_E_INVAL;
    }
    const SessReq &r = *it->second;
    *done = (r.state == RQ_DONE) ? 1 : 0;
    if (r.state == RQ_FAILED || r.state == RQ_CANCELLED) {
        set_error("ticket %llu ended with status %d", (unsigned long long)ticket, r.status);
        return r.status;
    }
    return FRG_OK;
}

frg_status frg_session_wait(frg_session *s, uint64_t ticket, int timeout_ms) {
    clear_error();
    if (!s) {
        set_error("null session");
        return FRG_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return FRG_E_INVAL;
    }
    SessReq *r = it->second.get();
    auto terminal = [&] { return r->state == RQ_DONE || r->state == RQ_FAILED ||
                                 r->state == RQ_CANCELLED; };
    if (timeout_ms < 0)
        s->cv.wait(lk, terminal);
    else if (!s->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), terminal)) {
        set_error("ticket %llu not finished after %d ms", (unsigned long long)ticket, timeout_ms);
        return FRG_E_TIMEOUT;
    }
    if (r->state != RQ_DONE) {
        set_error("ticket %llu ended with status %d", (unsigned long long)ticket, r->status);
        return r->status;
    }
    return FRG_OK;
}

frg_status frg_session_cancel(frg_session *s, uint64_t ticket) {
    clear_error();
    if (!s) {
        set_error("null session");
        return FRG_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return FRG_E_INVAL;
    }
    SessReq *r = it->second.get();
    if (r->state != RQ_QUEUED) {
        set_error("ticket %llu is already running or finished", (unsigned long long)ticket);
        return FRG_E_NOTREADY;
    }
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
    r->state = RQ_CANCELLED;
    r->status = FRG_E_CANCELLED;
    s->cancelled++;
    s->cv.notify_all();
    return FRG_OK;
}

frg_status frg_session_stats(frg_session *s, frg_stats *out) {
    clear_error();
    if (!s || !out) {
        set_error("null argument");
        return FRG_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof *out);
    std::vector<double> v = s->lat_us;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(p * v.size()) - 1);
            return v[i];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
    }
    double span = s->t_last - s->t_first;
    out->gnodes_per_s = span > 0 ? (double)s->nodes_done / (span * 1e-6) / 1e9 : 0.0;
    out->admitted = s->admitted;
    out->queued = s->queue.size();
    out->rejected = s->rejected;
    out->completed = s->completed;
    out->failed = s->failed;
    out->cancelled = s->cancelled;
    out->nodes = s->nodes_done;
    out->launches = s->launches;
    return FRG_OK;
}

frg_status frg_session_close(frg_session *s) {
    clear_error();
    if (!s) return FRG_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->thr.joinable()) s->thr.join();
    if (s->ctx) (void)hipSetDevice(s->ctx->device);
    delete s;
    return FRG_OK;
}

}  // extern "C"
