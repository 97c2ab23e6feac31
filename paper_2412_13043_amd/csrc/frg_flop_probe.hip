// FP64 FLOP count of the elementary sequences the integrand loops use, for the roofline's
// per-node work: one kernel per sequence runs it `iters` times per lane on a varying argument,
// and the hardware FP64 FLOP counter of each dispatch (read by a profiler) divided by the
// evaluations gives its FLOPs per call, after subtracting the same loop without the sequence.
#include "../../include/frg_testing.h"
#include "frg_internal.hpp"
#include "frg_math.hpp"

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

}  // namespace frg

using namespace frg;

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
