// Batched integration without any device allocation: frg_integrate_batch with its scratch in one
// static device array instead of the context's per-stream buffers.
//
// The scratch holds, in this order (each part 256-byte aligned):
//   - the descriptor's quadrature rules, only when the context has not cached them yet (built
//     on the caller's stream with the cache's kernels, so they carry the same values);
//   - the [n_q][n_ext] contribution block of radially chunked requests;
//   - the float32 form's per-point amplification slots, cleared by a fill kernel on every call
//     (no memset node, so the call can be captured into a HIP graph).
// The array is one per device and shared by every call on that device: it keeps the last
// call's contents, and calls whose work overlaps on one device (two streams, or two host
// threads) race on it.  Results are bitwise those of frg_integrate_batch: the same tile shape,
// request and kernels, only the scratch pointers differ.
#include <mutex>

#include "frg_runtime.hpp"

namespace frg {

constexpr size_t kNoAllocScratchBytes = FRG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// File-scope device array.  In host code its name is only a stand-in for the device symbol:
// kernels and copies get the address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

frg_status noalloc_scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d beyond the %d devices the static scratch table covers", device,
                  kMaxDevices);
        return FRG_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        FRG_HIP_CHECK(hipSetDevice(device));
        void *p = nullptr;
        FRG_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned no address for the static scratch");
            return FRG_E_DEVICE;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return FRG_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace frg

using namespace frg;

extern "C" frg_status frg_integrate_batch_noalloc(frg_context *ctx, const frg_integral_desc *desc,
                                                  const frg_batch *batch, hipStream_t stream) {
    clear_error();
    if (!ctx) {
        set_error("context is NULL");
        return FRG_E_INVAL;
    }
    frg_status st = validate(desc, batch, true);
    if (st != FRG_OK) return st;
    if (batch->n_ext == 0) return FRG_OK;
    std::lock_guard<std::mutex> lk(ctx->mu);
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    if (!ctx->noalloc_scratch) {
        set_error("the context has no static scratch address");
        return FRG_E_DEVICE;
    }
    // the same shape frg_integrate_batch chooses (results do not depend on it, speed does)
    const TileShape shape = choose_shape(ctx, *desc, batch->n_ext, 16 * ctx->num_cus);
    RadialRule rad{};
    AngleRule ang{};
    PhiRule phi{};
    const bool cached = cached_rules(ctx, *desc, &rad, &ang, &phi);
    ReqDev r;
    if ((st = make_request(ctx, *desc, *batch, shape, 1, 0.0, 1.0, &r, &rad, &ang, &phi)) !=
        FRG_OK)
        return st;
    const size_t rule_bytes = cached ? 0 : align256(rules_bytes(*desc));
    const size_t contrib_bytes = align256(contrib_doubles(r) * sizeof(double));
    const size_t ctr = (size_t)counter_count(r);
    const size_t need = rule_bytes + contrib_bytes + align256(ctr * sizeof(unsigned));
    if (need > kNoAllocScratchBytes) {
        set_error("this request needs %zu bytes of scratch (quadrature rules %zu, contributions "
                  "%zu), more than the %zu-byte static scratch of the no-allocation entry point",
                  need, rule_bytes, contrib_bytes, kNoAllocScratchBytes);
        return FRG_E_NOMEM;
    }
    char *base = (char *)ctx->noalloc_scratch;
    if (!cached &&
        (st = rules_into(ctx, *desc, base, rule_bytes, &r.rad, &r.ang, &r.phi, stream)) != FRG_OK)
        return st;
    double *contrib = (double *)(base + rule_bytes);
    unsigned *counters = (unsigned *)(base + rule_bytes + contrib_bytes);
    // the float32 slots must start at zero; the array keeps whatever the last call left
    FRG_HIP_CHECK(launch_fill_zero_u32(counters, ctr, stream));
    r.contrib_base = 0;
    r.ctr_base = 0;
    FRG_HIP_CHECK(launch_batch(&r, nullptr, tile_count(r), lds_bytes_for(r), contrib, counters,
                               stream));
    FRG_HIP_CHECK(launch_finalize(r, contrib, counters, stream));
    if (batch->dout_dz) FRG_HIP_CHECK(launch_dz(r, batch->dout_dz, stream));
    return FRG_OK;
}
