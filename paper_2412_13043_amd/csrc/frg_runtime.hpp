// Host runtime internals shared by the C-ABI entry points and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/frg.h"
#include "frg_internal.hpp"

namespace frg {

void set_error(const char *fmt, ...);
void clear_error();

#define FRG_HIP_CHECK(expr)                                                                   \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) {                                                               \
            ::frg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                             __LINE__);                                                       \
            return FRG_E_DEVICE;                                                              \
        }                                                                                     \
    } while (0)

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer &) = delete;
    DeviceBuffer &operator=(const DeviceBuffer &) = delete;
    ~DeviceBuffer() {
        if (ptr) (void)hipFree(ptr);
    }
    hipError_t alloc(size_t n) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, n > 0 ? n : 1);
        if (e == hipSuccess) {
            ptr = p;
            bytes = n;
        }
        return e;
    }
};

struct RadialEntry {
    DeviceBuffer buf;
    RadialRule rule;
};
struct AngleEntry {
    DeviceBuffer buf;
    AngleRule rule;
};
struct PhiEntry {
    DeviceBuffer buf;
    PhiRule rule;
};

// Per-stream scratch: contribution blocks, float32 amplification slots, work counters, and the
// request/tile tables of fused launches.  The amplification slots are zero at rest (the finalize
// kernel resets them after reading); the fused kernel's tile counter is cleared by a fill kernel
// before each launch.
struct Scratch {
    DeviceBuffer contrib;   // doubles (radially chunked requests)
    DeviceBuffer counters;  // u32, zero at rest
    DeviceBuffer work;      // 2 x u32: fused-launch tile counter
    DeviceBuffer reqs;      // ReqDev[]
    DeviceBuffer tiles;     // TileDev[]
    // pinned staging for the request/tile tables of fused launches; `staged` is recorded after
    // the upload so the staging area is not rewritten while a copy may still read it
    void *host_stage = nullptr;
    size_t host_bytes = 0;
    hipEvent_t staged = nullptr;
    // last fused call on this stream: its argument bytes and launch shape (plan cache)
    std::vector<char> last_key;
    int last_tiles = 0, last_grid = 0, last_lds = 0, last_nreqs = 0, last_fam = -1, last_prec = -1,
        last_reg = -1, last_der = -1, last_fin = 0;
    // and its dressing-table derivative blocks, launched after the integrals
    std::vector<std::pair<ReqDev, double *>> last_dz;
    ~Scratch() {
        if (host_stage) (void)hipHostFree(host_stage);
        if (staged) (void)hipEventDestroy(staged);
    }
};

// Tile shape of one request for the vertex families (the LPA family always uses lanes = points).
struct TileShape {
    int lq_log2 = 0;  // lanes per point over radial nodes (log2)
    int chunks = 1;   // radial chunks (separate workgroups) per external tile
    int lx_log2 = 0;  // lanes per point over cos1 nodes (log2; vertex families)
};

struct FlowGraph;

// Families by what they read: vertex families take external momenta and a dressing table.
inline bool is_vertex(int fam) {
    return fam == FRG_FAMILY_TWO_POINT || fam == FRG_FAMILY_THREE_POINT ||
           fam == FRG_FAMILY_TWO_POINT_T || fam == FRG_FAMILY_THREE_POINT_T;
}
inline bool is_ft(int fam) {
    return fam == FRG_FAMILY_LPA_T || fam == FRG_FAMILY_TWO_POINT_T ||
           fam == FRG_FAMILY_THREE_POINT_T;
}
inline bool is_lpa(int fam) { return fam == FRG_FAMILY_LPA || fam == FRG_FAMILY_LPA_T; }
// three-point families: a phi rule next to the cos1 rule
inline bool has_phi(int fam) {
    return fam == FRG_FAMILY_THREE_POINT || fam == FRG_FAMILY_THREE_POINT_T;
}
// doubles of the ext array for n points (real external frequencies)
inline long long ext_values(int fam, long long n) {
    if (fam == FRG_FAMILY_THREE_POINT_T) return 4 * n;
    if (fam == FRG_FAMILY_THREE_POINT || fam == FRG_FAMILY_TWO_POINT_T) return 2 * n;
    return fam == FRG_FAMILY_TWO_POINT ? n : 0;
}
// ... of a descriptor: complex external frequencies append their imaginary parts
inline long long ext_values(const frg_integral_desc &d, long long n) {
    if (d.complex_freq) return d.family == FRG_FAMILY_THREE_POINT_T ? 6 * n : 3 * n;
    return ext_values(d.family, n);
}
// doubles of the out array for n points (Re then Im with complex frequencies)
inline long long out_values(const frg_integral_desc &d, long long n) {
    return d.complex_freq ? 2 * n : n;
}
// kernel families (ReqDev::family) with a phi rule
inline bool req_has_phi(int fam) { return has_phi(fam) || fam == kFamThreePointComplex; }

// Matsubara frequency rule of a finite-temperature descriptor: frequencies 2 pi T (n + eta) for
// n = n_lo .. n_lo + n_exp - 1 (every |w| <= Lambda), and n_tail tail nodes per side beyond
// Omega; n_f = n_exp + 2 n_tail.
struct FreqRule {
    int n_f = 0, n_exp = 0, n_lo = 0, n_tail = 0;
    double eta = 0.0, T = 0.0, Omega = 0.0, lambda = 0.0;
};
frg_status freq_rule(const frg_integral_desc &d, FreqRule *out);
// The descriptor as planning sees it: a finite-temperature family as its vacuum counterpart
// (LPA or two-point) with n_q n_f radial nodes.  Other descriptors are returned unchanged.
frg_integral_desc plan_desc(const frg_integral_desc &d);
// Integrand nodes per external point.
double nodes_per_point(const frg_integral_desc &d);
// Order N of a polynomial-exponential regulator (0 for the other regulators).
int reg_order(const frg_integral_desc &d);
// y beyond which the order-n polynomial-exponential regulator is exactly 0 in float64.
double poly_exp_far_y(int n, double s_far);

}  // namespace frg

struct frg_context {
    int device = 0;
    size_t hbm_budget = 0;
    int num_cus = 256;
    std::mutex mu;
    hipStream_t aux = nullptr;  // rule construction and graph capture
    frg::DeviceBuffer logtab;   // float64 logarithm table (double2[256])
    frg::DeviceBuffer ones;     // {1, 1}: dressing table of requests without one
    // radial rules by (n, q_max, d, regulator, order)
    std::map<std::tuple<int, double, int, int, int>, std::unique_ptr<frg::RadialEntry>> radial;
    std::map<int, std::unique_ptr<frg::AngleEntry>> cos1;  // key n (+ 1 << 20: d = 3 weights)
    // finite-temperature radial rules by (n_q, q_max, k, T, Lambda, statistics, n_tail,
    // regulator and order)
    std::map<std::tuple<int, double, double, double, double, int, int, int>,
             std::unique_ptr<frg::RadialEntry>>
        ft_radial;
    std::map<int, std::unique_ptr<frg::PhiEntry>> phi;
    std::map<hipStream_t, std::unique_ptr<frg::Scratch>> scratch;
    std::map<std::vector<long long>, std::unique_ptr<frg::FlowGraph>> graphs;  // flow RHS plans
    bool flow_graphs = false;  // replay flow RHS plans as captured HIP graphs (FRG_FLOW_GRAPH=1)
    std::map<std::vector<int>, frg::TileShape> tuned;  // autotuned shapes (loaded/saved on disk)
    std::string tune_path;
    void *noalloc_scratch = nullptr;  // this device's static scratch (frg_integrate_batch_noalloc)
};

namespace frg {

// Validate a descriptor/batch pair; FRG_E_INVAL with a message on failure.
frg_status validate(const frg_integral_desc *desc, const frg_batch *batch, bool device_ptrs);
// Fill a ReqDev for a validated request (rules resolved through the context cache).
// rad, ang and phi (optional) replace the cached rules (a stepper's own finite-temperature
// rule; rules built outside the cache).
frg_status make_request(frg_context *ctx, const frg_integral_desc &desc, const frg_batch &b,
                        const TileShape &shape, int m2_mode, double m2_floor, double coef,
                        ReqDev *out, const RadialRule *rad = nullptr,
                        const AngleRule *ang = nullptr, const PhiRule *phi = nullptr);
// Finite-temperature radial rule of d written into buf (n_q n_f (4 doubles + 3 floats)), on
// stream s; *out points into buf.  base (optional): the d = 3 vacuum rule it is built from
// (default: the cached one).
frg_status ft_rule_into(frg_context *ctx, const frg_integral_desc &d, void *buf, size_t bytes,
                        RadialRule *out, hipStream_t s, const RadialRule *base = nullptr);
size_t ft_rule_bytes(int n_q, int n_f);
// Every rule of a descriptor from the context's cache, without building or allocating
// anything: false if one of them is not cached yet.
bool cached_rules(frg_context *ctx, const frg_integral_desc &d, RadialRule *rad, AngleRule *ang,
                  PhiRule *phi);
// Bytes of every rule of a descriptor laid out by rules_into (0 for an invalid descriptor).
size_t rules_bytes(const frg_integral_desc &d);
// Build every rule of a descriptor into caller-owned device memory on stream s, with the kernels
// and layouts of the cache (identical values); nothing is allocated.
frg_status rules_into(frg_context *ctx, const frg_integral_desc &d, void *buf, size_t bytes,
                      RadialRule *rad, AngleRule *ang, PhiRule *phi, hipStream_t s);
// Device address of the no-allocation entry point's static scratch on `device` (looked up once
// per device, with that device current).
frg_status noalloc_scratch_address(int device, void **out);
// Where a tile shape is used: a request launched alone (radial chunks wherever the heuristic
// finds them worth a finalize launch), a fused launch (tuned shapes as tuned; the heuristic
// chunks only two-point requests whose wavefronts hold one point each), or a launch with no
// finalize pass (no chunks at all: sessions).
enum class ShapeUse { kRequest, kFused, kNoChunks };
// Tile shape for a request: the autotuned one if the context has it, else the heuristic.
TileShape choose_shape(frg_context *ctx, const frg_integral_desc &desc, int n_ext,
                       int target_waves, ShapeUse use = ShapeUse::kRequest);
TileShape heuristic_shape(const frg_integral_desc &desc, int n_ext, int target_waves,
                          bool allow_chunks = true, bool fused = false);
// Doubles of contribution scratch and counters a request needs.
size_t contrib_doubles(const ReqDev &r);
int counter_count(const ReqDev &r);
int tile_count(const ReqDev &r);
// Workgroups of the finalize launch a fused launch needs for this request (0 unless chunked).
int finalize_blocks(const ReqDev &r);
// Scratch for a stream, grown to at least the given sizes.
frg_status get_scratch(frg_context *ctx, hipStream_t s, size_t contrib_doubles, size_t counters,
                       size_t n_reqs, size_t n_tiles, Scratch **out);
// Launch helpers (caller holds ctx->mu).
frg_status run_batch(frg_context *ctx, ReqDev &r, hipStream_t s, Scratch *sc);
frg_status run_multi(frg_context *ctx, std::vector<ReqDev> &reqs, hipStream_t s, Scratch *sc,
                     int grid_waves);
frg_status relaunch_multi(Scratch *sc, hipStream_t s);
// Tiles of a fused launch in longest-first order, and the dynamic LDS bytes it needs.
// et_ranges (optional, one per request): only the external tiles [first, second) of each.
std::vector<TileDev> make_tiles(const std::vector<ReqDev> &reqs, int *lds_out,
                                const std::vector<std::pair<int, int>> *et_ranges = nullptr);
// Family, precision and regulator shared by all requests (all -1 if any differs), and whether
// any request asks for the mass derivative.
void common_kind(const std::vector<ReqDev> &reqs, int *fam, int *prec, int *reg, int *der);
int lds_bytes_for(const ReqDev &r);

}  // namespace frg
