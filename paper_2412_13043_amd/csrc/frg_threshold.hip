// Threshold functions of the flat regulator, one of the library's convenience functions for
// standard fRG setups (Sec. 5, opening overview; the flat regulator of the regulator list):
//   l_n^d(w) = (2/d) (n + [n == 0]) / (1 + w)^(n+1),
// the closed form of the LPA loop integral with R = (k^2 - q^2) Theta(k^2 - q^2): its radial
// integral runs over [0, k] only, where q^2 + R = k^2 and k dR/dk = 2 k^2, so
// I(m^2) = Omega_d/(2 pi)^d k^(d-2) l_1^d(m^2/k^2).  Evaluated elementwise on the device.
#include <hip/hip_runtime.h>

#include "frg_runtime.hpp"

namespace frg {
namespace {

__global__ void __launch_bounds__(256) litim_threshold_kernel(int d, int n,
                                                              const double *__restrict__ w,
                                                              double *__restrict__ out,
                                                              int count) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= count) return;
    const double r = 1.0 / (1.0 + w[i]);
    double p = r;
    for (int j = 0; j < n; ++j) p *= r;
    out[i] = (2.0 / (double)d) * (double)(n == 0 ? 1 : n) * p;
}

bool device_memory(const void *p) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace
}  // namespace frg

using namespace frg;

extern "C" {

frg_status frg_litim_threshold(int d, int n, const double *w, double *out, int count,
                               hipStream_t stream) {
    clear_error();
    if (d < 1 || d > 16 || n < 0 || n > 16 || count < 0) {
        set_error("frg_litim_threshold needs 1 <= d <= 16, 0 <= n <= 16 and count >= 0 "
                  "(got d = %d, n = %d, count = %d)", d, n, count);
        return FRG_E_INVAL;
    }
    if (count == 0) return FRG_OK;
    if (!w || !out || !device_memory(w) || !device_memory(out)) {
        set_error("frg_litim_threshold needs device arrays w and out");
        return FRG_E_INVAL;
    }
    hipLaunchKernelGGL(litim_threshold_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256),
                       0, stream, d, n, w, out, count);
    FRG_HIP_CHECK(hipGetLastError());
    return FRG_OK;
}

}  // extern "C"
