// Serving loop: continuous batching of loop-integral requests from many concurrent clients.
//
// Requests are queued by frg_session_submit.  A scheduler thread packs queued requests into one
// fused launch of the multi-request tile consumer on a free launch slot, and keeps up to
// max_inflight such launches on separate streams: requests that arrive while others run join
// the next launch as slots and memory free up, and their work overlaps on the device.
//
// Memory: each launch takes one block of the session's HBM arena (hbm_budget_bytes) holding
// everything it touches -- the tile counter, the request and tile tables, the requests' inputs,
// the float32 form's amplification slots, the outputs and, for radially chunked shapes, the
// [n_q][n_ext] contributions -- so admission is by device footprint: a launch is only formed
// while its block fits the arena.  One copy uploads the block's first part (tables, inputs, the
// zeroed counter and slots) from the slot's pinned staging, one copy brings the outputs back:
// a launch is upload, the fused kernel, the radial sums of chunked requests, download, event.
//
// Scheduling rules:
//   - a launch holds at most kLaunchNodes integrand nodes (a few tenths of a millisecond of the
//     chip), so small requests never queue behind a long launch for long;
//   - a larger request is cut into parts of whole external tiles (multiples of 64 points for
//     chunked shapes, whose radial sums run per block of 64 points), each part a launch share
//     of its own with its own copy of the request's inputs, at most kPartsInFlight at once;
//     every point is computed inside one tile, so the result does not depend on the cut;
//   - every request keeps the tile shape frg_integrate_batch gives it alone;
//   - small requests (at most kSmallNodes) are launched first, then large ones, each class in
//     arrival order and in launches of their own; large requests hold at most half the slots
//     (rounded up), so a small request arriving while large launches run finds a free slot;
//   - launches run one workgroup per tile (no persistent grid), so concurrent launches share the
//     CUs tile by tile and a new small launch starts as soon as any running tile ends;
//   - requests that fit may go ahead of an earlier one that does not fit the arena yet, at most
//     kMaxBypass times per blocked request;
//   - pinned staging is allocated when the session opens; launching allocates nothing.
// Each result is computed exactly as frg_integrate_batch would compute it (results do not depend
// on batch composition, tile shape or the cut into parts).
//
// Execution goes through an Executor interface: the HIP executor, and a test double that runs
// no device work and completes a launch after a delay proportional to its node count, used by
// CPU-only tests of admission, splitting, cancellation, time-outs and accounting.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
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

constexpr size_t kMaxLaunchReqs = 512;       // requests (or parts) per launch
constexpr size_t kMaxLaunchTiles = 1 << 17;  // tiles (and radial-sum blocks) per launch
constexpr double kLaunchNodes = 2.0e8;       // integrand nodes per launch (~0.35 ms)
constexpr int kPartsInFlight = 2;            // parts of one request launched at once
constexpr int kMaxBypass = 64;               // admissions ahead of a request blocked on memory
constexpr double kSmallNodes = 1.0e8;        // small requests: scheduled first (~0.2 ms alone)
constexpr size_t kCounterBytes = 256;        // the fused kernel's tile counter, at block start

enum ReqState { RQ_QUEUED = 0, RQ_RUNNING, RQ_DONE, RQ_FAILED, RQ_CANCELLED };

struct SessReq {
    uint64_t ticket = 0;
    frg_integral_desc desc{};
    frg_batch host{};    // host pointers from the client
    int table_id = -1;
    int n_ext_vals = 0;  // doubles in ext
    int dz_n = 0;        // dressing-table entries per point of the dout_dz block (0: none)
    // inputs as laid out in a launch block (byte offsets from the part's input area): ext, m2,
    // the request's own dressing table
    size_t in_ext = 0, in_m2 = 0, in_z = 0, in_bytes = 0;
    size_t slot_bytes = 0;     // float32 amplification slots of a chunked shape (n_ext + 1)
    size_t contrib_bytes = 0;  // [n_q][n_ext] contributions of a chunked shape
    size_t footprint = 0;      // device bytes of the whole request in one launch (no tables)
    uint64_t nodes = 0;
    double t_submit = 0.0, t_done = 0.0;
    ReqState state = RQ_QUEUED;
    frg_status status = FRG_OK;
    bool timed_out = false;
    // tile shape (chosen at submit: the one frg_integrate_batch takes for the request alone),
    // its external tiles and the next one to launch; split: more than one launch's work
    TileShape shape{};
    bool split = false, chunked = false;
    int ext_tiles = 0, points_per_tile = 0, align_tiles = 1, next_et = 0, parts_inflight = 0;
    int bypassed = 0;  // admissions ahead of it while it could not be admitted
    // clients blocked in frg_session_wait on this ticket, and whether one of them (or a poll)
    // has been told the outcome (the ticket is forgotten once nothing refers to it any more)
    int waiters = 0;
    bool reported = false;
    std::condition_variable cv;
    bool terminal() const { return state == RQ_DONE || state == RQ_FAILED || state == RQ_CANCELLED; }
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
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }

   private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

// One request's share of a launch: its external tiles [et0, et1), points [p0, p1), and where
// its inputs, slots, outputs and contributions sit in the launch block (byte offsets).
struct Part {
    SessReq *r = nullptr;
    int et0 = 0, et1 = 0;
    int p0 = 0, p1 = 0;
    size_t in = 0, slots = 0, out = 0, contrib = 0;
    frg_log_table resident{};  // the session-resident dressing table, if the request uses one
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *host = nullptr;  // pinned staging of the launch block's uploaded and downloaded parts
    size_t host_bytes = 0;
    std::vector<Part> parts;
    // the launch block: arena offset and size; its layout (tables, then the parts' inputs and
    // slots = the upload, then their outputs = the download, then contributions)
    size_t block_off = (size_t)-1, block_bytes = 0;
    size_t tables_bytes = 0, upload_bytes = 0, out_begin = 0, out_end = 0;
    int n_tiles = 0;
    bool large = false;  // holds a part of a request above kSmallNodes
    bool busy = false;   // a launch is assigned (planned, running or being completed)
    bool assigned = false;  // planned, not yet picked up by the slot's worker
    double t_plan = 0.0, t_launch = 0.0, t_enqueued = 0.0;
    double fake_ready = 0.0;  // test double: completion time
    std::thread worker;
    std::condition_variable cv;  // the worker: a launch is assigned, or the session closes
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

// Latency histogram: logarithmic bins of 0.5 % from 0.1 us to 1e9 us (bounded memory; the
// percentiles are exact to the bin width).
class LatencyHist {
   public:
    static constexpr int kBins = 4400;
    static constexpr double kLo = 0.1;
    static constexpr double kStep = 1.005;
    void add(double us) {
        int b = us <= kLo ? 0 : (int)(std::log(us / kLo) / std::log(kStep)) + 1;
        b = std::min(std::max(b, 0), kBins - 1);
        ++bins_[b];
        ++n_;
    }
    // upper edge of the bin holding the p-quantile
    double quantile(double p) const {
        if (n_ == 0) return 0.0;
        const uint64_t want = (uint64_t)std::max(1.0, std::ceil(p * (double)n_));
        uint64_t c = 0;
        for (int b = 0; b < kBins; ++b) {
            c += bins_[b];
            if (c >= want) return kLo * std::pow(kStep, b);
        }
        return kLo * std::pow(kStep, kBins - 1);
    }

   private:
    uint64_t bins_[kBins] = {};
    uint64_t n_ = 0;
};

class Executor {
   public:
    virtual ~Executor() = default;
    virtual frg_status setup(frg_session &) = 0;
    // enqueue the slot's launch; called without the session lock
    virtual frg_status launch(frg_session &, Slot &) = 0;
    virtual int poll(frg_session &, Slot &) = 0;  // 1 done, 0 running, -1 device error
    virtual void finish(frg_session &, Slot &) = 0;
    // after a failed launch: wait until nothing queued on the slot's stream can still touch its
    // staging or its launch block
    virtual void drain(Slot &) = 0;
};

}  // namespace frg

struct frg_session {
    frg_context *ctx = nullptr;
    frg_session_config cfg{};
    std::unique_ptr<frg::Executor> exec;
    std::mutex mu;
    std::condition_variable sched_cv;  // the scheduler: new work, close
    std::thread thr;
    bool stop = false;
    std::deque<frg::SessReq *> queue;  // requests with tiles not yet launched
    std::unordered_map<uint64_t, std::unique_ptr<frg::SessReq>> reqs;
    uint64_t next_ticket = 1;
    frg::Arena arena;
    frg::DeviceBuffer arena_mem;
    size_t staging_bytes = 0;  // per slot
    std::vector<std::unique_ptr<frg::Slot>> slots;
    std::vector<std::unique_ptr<frg::ResidentTable>> tables;
    double fake_ns_per_node = 0.0, fake_base_us = 0.0;
    bool fake = false;
    std::atomic<int> fake_fail{0};  // test double: launches still to fail
    // statistics
    frg::LatencyHist lat;
    uint64_t admitted = 0, rejected = 0, completed = 0, failed = 0, cancelled = 0, nodes_done = 0,
             launches = 0;
    // per completed request: submit -> its last launch planned, planned -> enqueued on the
    // device, enqueued -> seen complete, seen complete -> result in the client's buffer
    double sum_queue_us = 0.0, sum_launch_us = 0.0, sum_device_us = 0.0, sum_finish_us = 0.0;
    double t_first = 0.0, t_last = 0.0;
    std::string fatal;
};

namespace frg {

// Points covered by external tiles [et0, et1) of a request.
static void part_points(const SessReq &r, int et0, int et1, int *p0, int *p1) {
    *p0 = std::min(et0 * r.points_per_tile, r.host.n_ext);
    *p1 = std::min(et1 * r.points_per_tile, r.host.n_ext);
}

// Output arrays a request returns: the integrals, then the float32 form's bounds and the mass
// derivatives if asked for, each [n] doubles in that order.
// arrays of a part's output area, each of its points: out (Re and Im with complex
// frequencies), err_out, dout_dm2
static int out_arrays(const SessReq &r) {
    return 1 + (r.desc.complex_freq ? 1 : 0) + (r.host.err_out ? 1 : 0) +
           (r.host.dout_dm2 ? 1 : 0);
}

// a part's output area: the out_arrays arrays of its points, then their dout_dz rows
static size_t part_out_bytes(const SessReq &r, int p0, int p1) {
    return align256((out_arrays(r) + (size_t)r.dz_n) * (size_t)(p1 - p0) * sizeof(double));
}

static size_t tables_bytes(size_t n_parts, size_t n_tiles) {
    return kCounterBytes + align256(n_parts * sizeof(ReqDev)) + align256(n_tiles * sizeof(TileDev));
}

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
            FRG_HIP_CHECK(hipHostMalloc(&sl->host, s.staging_bytes, hipHostMallocDefault));
            sl->host_bytes = s.staging_bytes;
        }
        return FRG_OK;
    }

    frg_status launch(frg_session &s, Slot &sl) override {
        frg_context *ctx = s.ctx;
        char *blk = (char *)s.arena_mem.ptr + sl.block_off;  // device launch block
        char *h = (char *)sl.host;                           // its staging on the host
        std::vector<ReqDev> rd;
        std::vector<std::pair<int, int>> ranges;
        // the context lock only for the requests' rules (the cache); the slot's own stream,
        // staging and block need no lock
        std::unique_lock<std::mutex> ctx_lk(ctx->mu);
        for (const Part &pt : sl.parts) {
            SessReq *r = pt.r;
            frg_batch b = r->host;
            const char *in = blk + pt.in;
            b.ext = is_vertex(r->desc.family) ? (const double *)(in + r->in_ext) : nullptr;
            b.m2 = r->host.m2 ? (const double *)(in + r->in_m2) : nullptr;
            // outputs of points [p0, p1) land at the part's output area
            b.out = (double *)(blk + pt.out) - pt.p0;
            const int ncx = r->desc.complex_freq ? 2 : 1;  // Re (and Im) come first
            b.err_out = r->host.err_out
                            ? (double *)(blk + pt.out) + ncx * (pt.p1 - pt.p0) - pt.p0
                            : nullptr;
            b.dout_dm2 = r->host.dout_dm2 ? (double *)(blk + pt.out) +
                                                (out_arrays(*r) - 1) * (pt.p1 - pt.p0) - pt.p0
                                          : nullptr;
            if (r->table_id >= 0)
                b.Z = pt.resident;
            else if (r->host.Z.values)
                b.Z.values = (const double *)(in + r->in_z);
            ReqDev q;
            frg_status st = make_request(ctx, r->desc, b, r->shape, 1, 0.0, 1.0, &q);
            if (st != FRG_OK) return st;
            // complex frequencies: Im of points [p0, p1) right after their Re in the area
            if (r->desc.complex_freq) q.dout = (double *)(blk + pt.out) + (pt.p1 - pt.p0) - pt.p0;
            // contributions and slots in the block, addressed from the block's start
            q.contrib_base = (long long)(pt.contrib / sizeof(double));
            q.ctr_base = (long long)(pt.slots / sizeof(unsigned));
            rd.push_back(q);
            ranges.emplace_back(pt.et0, pt.et1);
        }
        ctx_lk.unlock();
        int lds = 0;
        std::vector<TileDev> tiles = make_tiles(rd, &lds, &ranges);
        const size_t n_work = tiles.size();
        // radial sums of the chunked parts: one entry per block of 64 points (parts of chunked
        // requests start at multiples of 64 points)
        for (size_t i = 0; i < sl.parts.size(); ++i) {
            const Part &pt = sl.parts[i];
            if (!pt.r->chunked) continue;
            for (int b = pt.p0 / kWave; b * kWave < pt.p1; ++b)
                tiles.push_back(TileDev{(int)i, b, 0, 0});
        }
        const int n_fin = (int)(tiles.size() - n_work);
        if ((int)tiles.size() != sl.n_tiles) {
            set_error("internal: launch planned for %d tiles, built %zu", sl.n_tiles, tiles.size());
            return FRG_E_INVAL;
        }
        // upload area: counter (zero) | request table | tile table | inputs and zeroed slots
        const size_t reqs_off = kCounterBytes;
        const size_t tiles_off = reqs_off + align256(rd.size() * sizeof(ReqDev));
        std::memset(h, 0, kCounterBytes);
        std::memcpy(h + reqs_off, rd.data(), rd.size() * sizeof(ReqDev));
        std::memcpy(h + tiles_off, tiles.data(), tiles.size() * sizeof(TileDev));
        for (const Part &pt : sl.parts) {
            SessReq *r = pt.r;
            char *in = h + pt.in;
            if (is_vertex(r->desc.family))
                std::memcpy(in + r->in_ext, r->host.ext, (size_t)r->n_ext_vals * 8);
            if (r->host.m2) std::memcpy(in + r->in_m2, r->host.m2, (size_t)r->host.n_ext * 8);
            if (r->table_id < 0 && r->host.Z.values && is_vertex(r->desc.family))
                std::memcpy(in + r->in_z, r->host.Z.values, (size_t)r->host.Z.n * 8);
            if (r->slot_bytes) std::memset(h + pt.slots, 0, r->slot_bytes);
        }
        FRG_HIP_CHECK(hipMemcpyAsync(blk, h, sl.upload_bytes, hipMemcpyHostToDevice, sl.stream));
        const ReqDev *reqs_dev = (const ReqDev *)(blk + reqs_off);
        const TileDev *tiles_dev = (const TileDev *)(blk + tiles_off);
        int fam, prec, reg, der;
        common_kind(rd, &fam, &prec, &reg, &der);
        // one workgroup per tile: the launches of the slots interleave on the CUs tile by
        // tile, so a small launch starts while large ones run (a persistent grid would hold
        // its CU slots until its whole tile list is done)
        const int grid = (int)n_work;
        FRG_HIP_CHECK(launch_multi(reqs_dev, fam, prec, reg, der, tiles_dev, (int)n_work, grid,
                                   lds, (double *)blk, (unsigned *)blk, (unsigned *)blk,
                                   sl.stream, false));
        FRG_HIP_CHECK(launch_multi_finalize(reqs_dev, tiles_dev + n_work, n_fin,
                                            (const double *)blk, (unsigned *)blk, sl.stream));
        // dressing derivatives of the parts that ask for them, rows after the part's outputs
        for (size_t i = 0; i < sl.parts.size(); ++i) {
            const Part &pt = sl.parts[i];
            if (!pt.r->dz_n) continue;
            double *jac = (double *)(blk + pt.out) + (size_t)out_arrays(*pt.r) * (pt.p1 - pt.p0);
            FRG_HIP_CHECK(launch_dz_points(rd[i], jac, pt.p0, pt.p1 - pt.p0, sl.stream));
        }
        FRG_HIP_CHECK(hipMemcpyAsync(h + sl.out_begin, blk + sl.out_begin,
                                     sl.out_end - sl.out_begin, hipMemcpyDeviceToHost,
                                     sl.stream));
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
        for (const Part &pt : sl.parts) {
            const SessReq *r = pt.r;
            if (r->timed_out || r->state != RQ_RUNNING) continue;
            const size_t n = (size_t)(pt.p1 - pt.p0);
            std::memcpy(r->host.out + pt.p0, h + pt.out, n * 8);
            const size_t ncx = r->desc.complex_freq ? 2 : 1;
            if (ncx == 2)
                std::memcpy(r->host.out + r->host.n_ext + pt.p0, h + pt.out + n * 8, n * 8);
            if (r->host.err_out)
                std::memcpy(r->host.err_out + pt.p0, h + pt.out + ncx * n * 8, n * 8);
            if (r->host.dout_dm2)
                std::memcpy(r->host.dout_dm2 + pt.p0, h + pt.out + (out_arrays(*r) - 1) * n * 8,
                            n * 8);
            if (r->dz_n)
                std::memcpy(r->host.dout_dz + (size_t)pt.p0 * r->dz_n,
                            h + pt.out + out_arrays(*r) * n * 8, n * (size_t)r->dz_n * 8);
        }
    }

    void drain(Slot &sl) override { (void)hipStreamSynchronize(sl.stream); }
};

// Test double: no device work; a launch completes after base + ns_per_node * nodes.
class FakeExecutor : public Executor {
   public:
    frg_status setup(frg_session &) override { return FRG_OK; }
    frg_status launch(frg_session &s, Slot &sl) override {
        int f = s.fake_fail.load();
        while (f > 0 && !s.fake_fail.compare_exchange_weak(f, f - 1)) {
        }
        if (f > 0) {
            set_error("test double: launch failure requested");
            return FRG_E_DEVICE;
        }
        double nodes = 0.0;
        for (const Part &pt : sl.parts)
            nodes += (double)(pt.p1 - pt.p0) * nodes_per_point(pt.r->desc);
        sl.fake_ready = now_us() + s.fake_base_us + s.fake_ns_per_node * nodes * 1e-3;
        return FRG_OK;
    }
    int poll(frg_session &, Slot &sl) override { return now_us() >= sl.fake_ready ? 1 : 0; }
    void finish(frg_session &, Slot &) override {}
    void drain(Slot &) override {}
};

// ---------------------------------------------------------------------------------------------
// Scheduler (every function below runs with s.mu held)
// ---------------------------------------------------------------------------------------------
// A ticket whose outcome a client has been told and that nothing refers to any more is dropped.
static void maybe_forget(frg_session &s, SessReq *r) {
    if (r->reported && r->waiters == 0 && r->terminal() && r->parts_inflight == 0)
        s.reqs.erase(r->ticket);
}

static void remove_from_queue(frg_session &s, SessReq *r) {
    auto it = std::find(s.queue.begin(), s.queue.end(), r);
    if (it != s.queue.end()) s.queue.erase(it);
}

static void end_request(frg_session &s, SessReq *r, ReqState state, frg_status status, double t) {
    if (r->terminal()) return;
    r->state = state;
    r->status = status;
    r->t_done = t;
    if (state == RQ_DONE) {
        s.completed++;
        s.nodes_done += r->nodes;
        s.lat.add(t - r->t_submit);
        s.t_last = t;
    } else if (state == RQ_FAILED) {
        s.failed++;
    } else {
        s.cancelled++;
    }
    r->cv.notify_all();
}

// Bookkeeping after a launch ended (outputs already copied to the clients' buffers if ok).
static void complete_slot(frg_session &s, Slot &sl, bool ok, double t_seen) {
    const double t = now_us();
    if (sl.block_off != Arena::npos) {
        s.arena.release(sl.block_off, sl.block_bytes);
        sl.block_off = Arena::npos;
    }
    for (const Part &pt : sl.parts) {
        SessReq *r = pt.r;
        r->parts_inflight--;
        if (!ok) {
            remove_from_queue(s, r);  // no further parts
            end_request(s, r, RQ_FAILED, FRG_E_DEVICE, t);
        }
        if (r->parts_inflight == 0 && (r->next_et >= r->ext_tiles || r->terminal()) &&
            !r->terminal()) {
            s.sum_queue_us += sl.t_plan - r->t_submit;
            s.sum_launch_us += sl.t_enqueued - sl.t_plan;
            s.sum_device_us += t_seen - sl.t_enqueued;
            s.sum_finish_us += t - t_seen;
            end_request(s, r, RQ_DONE, FRG_OK, t);
        }
        maybe_forget(s, r);
    }
    sl.parts.clear();
    sl.busy = false;
    s.sched_cv.notify_all();  // a slot and arena memory are free
}

// Choose the parts of one launch for a free slot and place them in one arena block; false if
// there is nothing to launch.  Small requests (at most kSmallNodes) go first, in arrival order,
// and a launch with small requests takes no large ones; large requests hold at most half the
// slots (rounded up), so a small request that arrives while large launches run finds a slot.
static bool plan_launch(frg_session &s, Slot &sl) {
    // room for one launch block: the arena's largest free range and the slot's staging
    const size_t room = s.arena.largest_free();
    int large_running = 0;
    for (const auto &x : s.slots)
        if (x->busy && x->large) ++large_running;
    const bool large_ok = large_running < std::max(1, ((int)s.slots.size() + 1) / 2);
    double nodes = 0.0;
    size_t n_tiles = 0, data = 0, upload_data = 0, out_data = 0;
    SessReq *blocked = nullptr;  // the earliest request that did not fit
    bool full = false, large = false;
    std::vector<SessReq *> done_launching;
    struct Pick {
        SessReq *r;
        int et0, et1, p0, p1;
    };
    std::vector<Pick> picks;
    for (int pass = 0; pass < 2 && !full; ++pass) {
        // a launch holds small requests or large ones, not both (a small request in a launch
        // with a large part would wait for the part)
        if (pass == 1 && (!large_ok || !picks.empty())) break;
        for (size_t qi = 0; qi < s.queue.size() && !full; ++qi) {
            if (picks.size() >= kMaxLaunchReqs) {
                full = true;
                break;
            }
            SessReq *r = s.queue[qi];
            if (((double)r->nodes > kSmallNodes) != (pass == 1)) continue;
            const bool started = r->next_et > 0;
            if (started && r->parts_inflight >= kPartsInFlight) continue;
            const double npp = nodes_per_point(r->desc);
            const int remaining = r->ext_tiles - r->next_et;
            const size_t per_tile = (size_t)r->shape.chunks;  // work tiles per external tile
            int k;
            if (!r->split) {
                if (!picks.empty() && nodes + (double)r->nodes > kLaunchNodes) {
                    full = true;
                    break;
                }
                k = remaining;
            } else {
                // as many whole tiles as the launch has room for, in multiples of align_tiles
                // (at least one multiple)
                const double tile_nodes = (double)r->points_per_tile * npp;
                const int a = r->align_tiles;
                k = (int)std::floor((kLaunchNodes - nodes) / tile_nodes);
                k = (int)std::min<long long>(k,
                                             (long long)((kMaxLaunchTiles - n_tiles) / per_tile));
                k = (k / a) * a;
                if (k < a) {
                    if (!picks.empty()) {
                        full = true;
                        break;
                    }
                    k = a;
                }
                k = std::min(k, remaining);
            }
            int p0, p1;
            part_points(*r, r->next_et, r->next_et + k, &p0, &p1);
            const size_t fin = r->chunked ? (size_t)(p1 - p0 + kWave - 1) / kWave : 0;
            const size_t pt_tiles = (size_t)k * per_tile + fin;
            const size_t up = align256(r->in_bytes) + align256(r->slot_bytes);
            const size_t down = part_out_bytes(*r, p0, p1);
            const size_t tb = tables_bytes(picks.size() + 1, n_tiles + pt_tiles);
            const size_t need_block = tb + data + up + down + align256(r->contrib_bytes);
            const size_t need_stage = tb + upload_data + up + out_data + down;
            if (n_tiles + pt_tiles > kMaxLaunchTiles || need_stage > s.staging_bytes) {
                if (!picks.empty()) {
                    full = true;
                    break;
                }
                continue;  // cannot happen for a request accepted at submit
            }
            if (need_block > room) {
                if (!picks.empty()) {
                    full = true;  // the launch is full
                    break;
                }
                // it does not fit the arena right now: later requests may go ahead of it, a
                // bounded number of times
                if (!blocked && !started) blocked = r;
                continue;
            }
            if (!started) {
                if (blocked && blocked->bypassed >= kMaxBypass) continue;
                r->state = RQ_RUNNING;
                s.admitted++;
                if (blocked) blocked->bypassed++;
            }
            picks.push_back(Pick{r, r->next_et, r->next_et + k, p0, p1});
            n_tiles += pt_tiles;
            data += up + down + align256(r->contrib_bytes);
            upload_data += up;
            out_data += down;
            nodes += (double)(p1 - p0) * npp;
            large = large || pass == 1;
            r->parts_inflight++;
            r->next_et += k;
            if (r->next_et >= r->ext_tiles) done_launching.push_back(r);
            if (nodes >= kLaunchNodes) full = true;
        }
    }
    for (SessReq *r : done_launching) remove_from_queue(s, r);
    if (picks.empty()) return false;
    sl.large = large;
    // block layout: tables | inputs and slots of every part (upload) | outputs (download) |
    // contributions
    const size_t tb = tables_bytes(picks.size(), n_tiles);
    size_t pos = tb;
    sl.parts.clear();
    for (const Pick &pk : picks) {
        Part pt;
        pt.r = pk.r;
        pt.et0 = pk.et0;
        pt.et1 = pk.et1;
        pt.p0 = pk.p0;
        pt.p1 = pk.p1;
        pt.in = pos;
        pos += align256(pk.r->in_bytes);
        pt.slots = pos;
        pos += align256(pk.r->slot_bytes);
        if (pk.r->table_id >= 0) {
            const ResidentTable &t = *s.tables[pk.r->table_id];
            pt.resident = frg_log_table{(const double *)t.buf.ptr, t.n, t.x_min, t.x_max};
        }
        sl.parts.push_back(pt);
    }
    sl.upload_bytes = pos;
    sl.out_begin = pos;
    for (Part &pt : sl.parts) {
        pt.out = pos;
        pos += part_out_bytes(*pt.r, pt.p0, pt.p1);
    }
    sl.out_end = pos;
    for (Part &pt : sl.parts) {
        pt.contrib = pos;
        pos += align256(pt.r->contrib_bytes);
    }
    sl.tables_bytes = tb;
    sl.n_tiles = (int)n_tiles;
    sl.block_bytes = pos;
    sl.block_off = s.arena.alloc(pos);  // fits: pos <= the largest free range
    return true;
}

// Assign the next launch to a free slot; false if no slot is free or nothing can be launched.
static bool plan_next(frg_session &s) {
    Slot *sl = nullptr;
    for (auto &x : s.slots)
        if (!x->busy) {
            sl = x.get();
            break;
        }
    if (!sl || s.queue.empty()) return false;
    if (!plan_launch(s, *sl)) return false;
    sl->busy = true;
    sl->assigned = true;
    sl->t_plan = now_us();
    s.launches++;
    sl->cv.notify_one();
    return true;
}

// The slot's worker: enqueue each assigned launch (without the session lock, so clients keep
// submitting and other slots keep launching), wait for it by polling its completion every
// poll_us (spinning: a sleep this short would last the kernel's timer slack, ~50 us, instead),
// copy the outputs to the clients' buffers and hand the slot back.
static void slot_worker(frg_session *sp, Slot *slp) {
    frg_session &s = *sp;
    Slot &sl = *slp;
    if (s.ctx) (void)hipSetDevice(s.ctx->device);
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
        sl.cv.wait(lk, [&] { return sl.assigned || (s.stop && !sl.busy); });
        if (!sl.assigned) return;
        sl.assigned = false;
        lk.unlock();
        frg_status st = s.exec->launch(s, sl);
        sl.t_enqueued = now_us();
        std::string msg = st == FRG_OK ? std::string() : std::string(frg_last_error());
        int p = st == FRG_OK ? 0 : -1;
        if (st != FRG_OK) s.exec->drain(sl);
        while (p == 0) {
            p = s.exec->poll(s, sl);
            if (p != 0) break;
            if (s.fake) {  // the test double's launches last milliseconds: no need to spin
                std::this_thread::sleep_for(std::chrono::microseconds(s.cfg.poll_us));
                continue;
            }
            const double until = now_us() + (double)s.cfg.poll_us;
            while (now_us() < until) std::this_thread::yield();
        }
        const double t_seen = now_us();
        if (p < 0 && st == FRG_OK) msg = frg_last_error();
        // outputs into the clients' buffers (their requests are running: nobody else touches
        // them); requests the watchdog already failed are skipped inside finish
        if (p > 0) {
            lk.lock();
            s.exec->finish(s, sl);
            complete_slot(s, sl, true, t_seen);
        } else {
            lk.lock();
            s.fatal = msg;
            complete_slot(s, sl, false, t_seen);
        }
    }
}

// The scheduler: forms launches whenever a slot is free and work is queued, and runs the
// watchdog over launches in flight.
static void scheduler(frg_session *sp) {
    frg_session &s = *sp;
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
        while (!s.stop && plan_next(s)) {
        }
        bool busy = false;
        for (auto &sl : s.slots) busy = busy || sl->busy;
        if (s.stop && !busy) break;
        if (s.cfg.watchdog_ms > 0 && busy) {
            const double now = now_us();
            for (auto &sl : s.slots) {
                if (!sl->busy || now - sl->t_plan <= 1e3 * s.cfg.watchdog_ms) continue;
                for (const Part &pt : sl->parts) {
                    SessReq *r = pt.r;
                    if (r->timed_out || r->terminal()) continue;
                    r->timed_out = true;
                    remove_from_queue(s, r);
                    end_request(s, r, RQ_FAILED, FRG_E_TIMEOUT, now);
                }
            }
            s.sched_cv.wait_for(lk, std::chrono::milliseconds(1));
        } else {
            s.sched_cv.wait(lk);
        }
    }
    // queued tickets left at close are cancelled (a split request may have launched parts)
    for (SessReq *r : s.queue) end_request(s, r, RQ_CANCELLED, FRG_E_CANCELLED, now_us());
    s.queue.clear();
    for (auto &sl : s.slots) sl->cv.notify_all();
}

// Inputs of a request as one launch block holds them, and its other device needs.
static void request_layout(SessReq &r) {
    const frg_integral_desc &d = r.desc;
    const size_t n = (size_t)r.host.n_ext;
    size_t off = 0;
    r.n_ext_vals = (int)ext_values(d, (long long)n);
    r.in_ext = off;
    off += (size_t)r.n_ext_vals * 8;
    r.in_m2 = off;
    if (r.host.m2) off += n * 8;
    r.in_z = off;
    if (r.table_id < 0 && r.host.Z.values && is_vertex(d.family)) off += (size_t)r.host.Z.n * 8;
    r.in_bytes = off;
    r.slot_bytes = (r.chunked && d.precision == FRG_FP32_KAHAN) ? (n + 1) * 4 : 0;
    // radial contributions of a chunked shape, and as many derivative contributions
    r.contrib_bytes =
        r.chunked ? (size_t)plan_desc(d).n_q * n * 8 * (r.host.dout_dm2 || d.complex_freq ? 2 : 1)
                  : 0;
    r.footprint = align256(r.in_bytes) + align256(r.slot_bytes) +
                  align256((out_arrays(r) + (size_t)r.dz_n) * n * 8) + align256(r.contrib_bytes);
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
    if (s->cfg.poll_us == 0) s->cfg.poll_us = 2;
    size_t budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (ctx ? ctx->hbm_budget : 0);
    if (budget < 4096) {
        set_error("session HBM budget must be at least 4096 bytes");
        return FRG_E_INVAL;
    }
    s->arena.init(budget & ~(size_t)255);
    s->staging_bytes = FRG_SESSION_STAGING_BYTES;
    for (int i = 0; i < cfg->max_inflight; ++i) s->slots.push_back(std::make_unique<Slot>());
    s->fake_ns_per_node = ns_per_node;
    s->fake_base_us = base_us;
    s->fake = fake;
    if (fake)
        s->exec = std::make_unique<FakeExecutor>();
    else
        s->exec = std::make_unique<HipExecutor>();
    frg_status st = s->exec->setup(*s);
    if (st != FRG_OK) return st;
    frg_session *raw = s.get();
    for (auto &sl : s->slots) sl->worker = std::thread(slot_worker, raw, sl.get());
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

frg_status frg_session_fake_fail_launches(frg_session *s, int n) {
    clear_error();
    if (!s || !s->fake || n < 0) {
        set_error("frg_session_fake_fail_launches needs a fake session and n >= 0");
        return FRG_E_INVAL;
    }
    s->fake_fail.store(n);
    return FRG_OK;
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
    if (!desc || !batch_host) {
        set_error("null descriptor or batch");
        return FRG_E_INVAL;
    }
    // a request on a resident table is checked against that table (dout_dz needs a table)
    frg_batch vb = *batch_host;
    int dz_n = batch_host->Z.values ? batch_host->Z.n : 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (table_id >= (int)s->tables.size() || table_id < -1) {
            set_error("unknown table id %d", table_id);
            return FRG_E_INVAL;
        }
        if (table_id >= 0) {
            // the resident table replaces the batch's (launches use it)
            const ResidentTable &t = *s->tables[table_id];
            vb.Z = frg_log_table{(const double *)&t, t.n, t.x_min, t.x_max};  // not read
            dz_n = t.n;
        }
    }
    frg_status st = validate(desc, &vb, false);
    if (st != FRG_OK) return st;
    auto r = std::make_unique<SessReq>();
    r->desc = *desc;
    r->host = *batch_host;
    r->table_id = table_id;
    r->dz_n = batch_host->dout_dz ? dz_n : 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            set_error("session is closing");
            return FRG_E_CANCELLED;
        }
    }
    const frg_integral_desc &d = *desc;
    const double npp = nodes_per_point(d);
    const int n = batch_host->n_ext;
    r->nodes = (uint64_t)((double)n * npp);
    // the tile shape frg_integrate_batch takes for the request alone (radial chunks included)
    const int target = 16 * (s->ctx ? s->ctx->num_cus : 256);
    if (s->ctx) {
        std::lock_guard<std::mutex> lk(s->ctx->mu);
        r->shape = choose_shape(s->ctx, d, std::max(n, 1), target, ShapeUse::kRequest);
    } else {
        r->shape = heuristic_shape(d, std::max(n, 1), target, true, false);
    }
    if (is_lpa(d.family)) r->shape = TileShape{};
    r->chunked = r->shape.chunks > 1;
    r->points_per_tile = is_lpa(d.family) ? kWave : (kWave >> (r->shape.lq_log2 + r->shape.lx_log2));
    r->ext_tiles = (n + r->points_per_tile - 1) / r->points_per_tile;
    r->align_tiles = r->chunked ? kWave / r->points_per_tile : 1;
    // parts when the request exceeds one launch's work or a good share of its tile table
    r->split = n > 0 && ((double)r->nodes > kLaunchNodes ||
                         (size_t)r->ext_tiles * r->shape.chunks > kMaxLaunchTiles / 2);
    request_layout(*r);
    // a launch of this request alone (its largest part): tables and the request's device bytes
    const size_t tiles_alone =
        std::min<size_t>((size_t)r->ext_tiles * r->shape.chunks +
                             (r->chunked ? ((size_t)n + kWave - 1) / kWave : 0),
                         kMaxLaunchTiles);
    const size_t alone = tables_bytes(1, tiles_alone) + r->footprint;
    const size_t alone_stage = alone - align256(r->contrib_bytes);
    r->t_submit = now_us();
    std::lock_guard<std::mutex> lk(s->mu);
    if (alone > s->arena.capacity()) {
        s->rejected++;
        set_error("request needs %zu device bytes, more than the session budget %zu", alone,
                  s->arena.capacity());
        return FRG_E_NOMEM;
    }
    if (alone_stage > s->staging_bytes) {
        s->rejected++;
        set_error("request needs %zu bytes of host staging, more than the %zu a launch slot has",
                  alone_stage, s->staging_bytes);
        return FRG_E_NOMEM;
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    if (s->t_first == 0.0) s->t_first = r->t_submit;
    SessReq *raw = r.get();
    s->reqs.emplace(r->ticket, std::move(r));
    if (batch_host->n_ext == 0) {
        end_request(*s, raw, RQ_DONE, FRG_OK, raw->t_submit);
    } else {
        s->queue.push_back(raw);
        s->sched_cv.notify_all();
    }
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
    SessReq *r = it->second.get();
    *done = (r->state == RQ_DONE) ? 1 : 0;
    if (!r->terminal()) return FRG_OK;
    const frg_status st = r->state == RQ_DONE ? FRG_OK : r->status;
    if (st != FRG_OK)
        set_error("ticket %llu ended with status %d", (unsigned long long)ticket, r->status);
    r->reported = true;
    maybe_forget(*s, r);
    return st;
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
    auto terminal = [&] { return r->terminal(); };
    r->waiters++;
    bool ended = true;
    if (timeout_ms < 0)
        r->cv.wait(lk, terminal);
    else
        ended = r->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), terminal);
    r->waiters--;
    if (!ended) {
        set_error("ticket %llu not finished after %d ms", (unsigned long long)ticket, timeout_ms);
        return FRG_E_TIMEOUT;
    }
    const frg_status st = r->state == RQ_DONE ? FRG_OK : r->status;
    if (st != FRG_OK)
        set_error("ticket %llu ended with status %d", (unsigned long long)ticket, r->status);
    r->reported = true;
    maybe_forget(*s, r);
    return st;
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
    remove_from_queue(*s, r);
    end_request(*s, r, RQ_CANCELLED, FRG_E_CANCELLED, now_us());
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
    out->p50_us = s->lat.quantile(0.50);
    out->p99_us = s->lat.quantile(0.99);
    double span = s->t_last - s->t_first;
    out->gnodes_per_s = span > 0 ? (double)s->nodes_done / (span * 1e-6) / 1e9 : 0.0;
    out->admitted = s->admitted;
    out->queued = 0;
    for (const SessReq *r : s->queue)
        if (r->state == RQ_QUEUED) out->queued++;
    out->rejected = s->rejected;
    out->completed = s->completed;
    out->failed = s->failed;
    out->cancelled = s->cancelled;
    out->nodes = s->nodes_done;
    out->launches = s->launches;
    out->tickets_held = s->reqs.size();
    if (s->completed) {
        const double c = (double)s->completed;
        out->mean_queue_us = s->sum_queue_us / c;
        out->mean_launch_us = s->sum_launch_us / c;
        out->mean_device_us = s->sum_device_us / c;
        out->mean_finish_us = s->sum_finish_us / c;
    }
    return FRG_OK;
}

frg_status frg_session_close(frg_session *s) {
    clear_error();
    if (!s) return FRG_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->sched_cv.notify_all();
    }
    if (s->thr.joinable()) s->thr.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &sl : s->slots) sl->cv.notify_all();
    }
    for (auto &sl : s->slots)
        if (sl->worker.joinable()) sl->worker.join();
    if (s->ctx) (void)hipSetDevice(s->ctx->device);
    delete s;
    return FRG_OK;
}

}  // extern "C"
