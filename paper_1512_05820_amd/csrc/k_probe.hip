// Bandwidth probe of libpodcg (podcg_stream_triad): not part of the method,
// it measures the streaming rate the loop kernels are compared with.
#include "podcg_launch.h"

namespace podcg {

// Stream triad c = a + s b: 16 bytes per lane, two elements of each thread in
// flight, nontemporal loads.  Measured on MI355X at 512 workgroups: with three
// 1 GB arrays (what the bench uses) 5.8 TB/s; with three 134 MB arrays, which
// the 256 MB last-level cache partly holds from one launch to the next,
// 7.1 TB/s with these loads against 5.8 TB/s with plain ones (and 5.0-5.6 TB/s
// with 8-byte lanes).  An odd last element is handled by one thread.
typedef double dbl2_t __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(kBlock) void k_triad(const double* __restrict__ a,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ c, size_t n, double s) {
    const size_t n2 = n / 2;
    const dbl2_t* __restrict__ a2 = (const dbl2_t*)a;
    const dbl2_t* __restrict__ b2 = (const dbl2_t*)b;
    dbl2_t* __restrict__ c2 = (dbl2_t*)c;
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n2; i += 2 * stride) {
        const size_t j = i + stride;
        const dbl2_t x0 = __builtin_nontemporal_load(a2 + i), y0 = __builtin_nontemporal_load(b2 + i);
        dbl2_t x1 = x0, y1 = y0;
        if (j < n2) {
            x1 = __builtin_nontemporal_load(a2 + j);
            y1 = __builtin_nontemporal_load(b2 + j);
        }
        c2[i] = x0 + s * y0;
        if (j < n2) c2[j] = x1 + s * y1;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) c[n - 1] = a[n - 1] + s * b[n - 1];
}

hipError_t launch_triad(const double* a, const double* b, double* c, size_t n, double sc,
                        hipStream_t s) {
    // 16-byte lanes need 16-byte aligned arrays
    if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return hipErrorInvalidValue;
    int64_t g = ((int64_t)n / 2 + kBlock - 1) / kBlock;
    if (g > 512) g = 512;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_triad, dim3((int)g), dim3(kBlock), 0, s, a, b, c, n, sc);
    return hipGetLastError();
}

}  // namespace podcg
