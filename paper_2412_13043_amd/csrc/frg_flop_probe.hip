// Probes of the elementary sequences the integrand loops use.
// FP64 FLOP count of the elementary sequences the integrand loops use, for the roofline's
// per-node work: one kernel per sequence runs it `iters` times per lane on a varying argument,
// and the hardware FP64 FLOP counter of each dispatch (read by a profiler) divided by the
// evaluations gives its FLOPs per call, after subtracting the same loop without the sequence.
#include "../../include/frg_testing.h"
#include "frg_internal.hpp"
#include "frg_math.hpp"

#include <cstring>

namespace frg {

// SEQ 0: the loop alone; 1: fm::log_tab; 2: fm::expm1_neg; 3: fm::exp_neg; 4: fm::rcp_nr.
template <int SEQ>
__global__ void __launch_bounds__(64) flop_probe_kernel(double *out, int iters,
                                                        const double2 *__restrict__ logt) {
    const int gid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    double x = 1.5 + 1e-3 * threadIdx.x + 1e-6 * blockIdx.x;
    double acc = 0.0;
    for (int i = 0; i < iters; ++i) {
        double v;
        if (SEQ == 1)
            v = fm::log_tab(x, logt);
        else if (SEQ == 2)
            v = fm::expm1_neg(x);
        else if (SEQ == 3)
            v = fm::exp_neg(x);
        else if (SEQ == 4)
            v = fm::rcp_nr(x);
        else
            v = x;
        acc += v;
        x += 0.0009765625;
    }
    out[gid] = acc;
}

// Accuracy of the float32 form's elementary operations, over every float32 input of a range
// (a grid-stride loop; each wavefront's largest error joins a device maximum):
//  0: |v_log_f32(m) - log2(m)| (absolute) for m in [1/2, 1)  (2^23 inputs);
//  1: |fm::expm1_neg_f(y) - expm1(-y)| / |expm1(-y)| for normal y in [2^-126, 2^21] (above that the
//     argument is clamped and the result is -1, off by e^-y);
//  2: |v_rcp_f32(d) d - 1| for d in [2^-100, 2^100);
//  3: |v_exp_f32(x) - 2^x| / 2^x for x in [-126, 0) (normal results).
// The references are the float64 log2, expm1 and exp2 of the HIP math library.
__global__ void __launch_bounds__(256) math_probe_kernel(int which, unsigned long long lo,
                                                         unsigned long long hi,
                                                         unsigned long long *maxbits) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    double worst = 0.0;
    for (unsigned long long b = lo + blockIdx.x * blockDim.x + threadIdx.x; b < hi; b += stride) {
        const float x = __uint_as_float((unsigned)b);
        double err;
        if (which == 0) {
            err = fabs((double)__builtin_amdgcn_logf(x) - log2((double)x));
        } else if (which == 1) {
            const double E = expm1(-(double)x);
            err = fabs((double)fm::expm1_neg_f(x) - E) / fabs(E);
        } else if (which == 2) {
            err = fabs((double)__builtin_amdgcn_rcpf(x) * (double)x - 1.0);
        } else {
            const double e = exp2((double)x);
            err = fabs((double)__builtin_amdgcn_exp2f(x) - e) / e;
        }
        worst = fmax(worst, err);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o));
    if ((threadIdx.x & (kWave - 1)) == 0)
        atomicMax(maxbits, (unsigned long long)__double_as_longlong(worst));
}

}  // namespace frg

using namespace frg;

extern "C" frg_status frg_math_probe(int which, double *max_err, hipStream_t stream) {
    if (which < 0 || which > 3 || !max_err) return FRG_E_INVAL;
    // input ranges as float32 bit patterns [lo, hi) (which 3: -0 excluded up to -126 included)
    const unsigned long long lo[4] = {0x3F000000ull, 0x00800000ull, 0x0D800000ull, 0x80000001ull};
    const unsigned long long hi[4] = {0x3F800000ull, 0x4A000001ull, 0x71800000ull, 0xC2FC0001ull};
    unsigned long long *d = nullptr;
    if (hipMalloc(&d, sizeof(unsigned long long)) != hipSuccess) return FRG_E_DEVICE;
    hipError_t e = hipMemsetAsync(d, 0, sizeof(unsigned long long), stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(math_probe_kernel, dim3(2048), dim3(256), 0, stream, which, lo[which],
                           hi[which], d);
        e = hipGetLastError();
    }
    unsigned long long bits = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bits, d, sizeof(bits), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(d);
    if (e != hipSuccess) return FRG_E_DEVICE;
    std::memcpy(max_err, &bits, sizeof(double));
    return FRG_OK;
}

extern "C" void frg_fp32_error_constants(double out[5]) {
    out[0] = kU32;
    out[1] = kErrLog2f;
    out[2] = kErrExpm1f;
    out[3] = kErrRcpf;
    out[4] = kErrExp2f;
}

extern "C" frg_status frg_flop_probe(int seq, int blocks, int iters, double *out,
                                     hipStream_t stream) {
    if (seq < 0 || seq > 4 || blocks < 1 || iters < 1 || !out) return FRG_E_INVAL;
    double2 *logt = nullptr;
    if (hipMalloc(&logt, kLogTable * sizeof(double2)) != hipSuccess) return FRG_E_DEVICE;
    hipError_t e = launch_log_table(logt, stream);
    void (*fn)(double *, int, const double2 *) =
        seq == 1 ? flop_probe_kernel<1>
                 : (seq == 2 ? flop_probe_kernel<2>
                             : (seq == 3 ? flop_probe_kernel<3>
                                         : (seq == 4 ? flop_probe_kernel<4> : flop_probe_kernel<0>)));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(kWave), 0, stream, out, iters, logt);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(logt);
    return e == hipSuccess ? FRG_OK : FRG_E_DEVICE;
}
