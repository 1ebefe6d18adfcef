// Estimators from the root counts R (Algorithm 1's last loop and the farness
// identity of Section 4.2):
//   diag[v]      = R[v] / tau                      estimates Omega_vv
//   farness[v]   = (n R[v] + S) / tau - 2          n Omega_vv + tr(Omega) - 2
//   closeness[v] = n / farness[v]
// with S = sum_w R[w] an exact 64-bit integer, so every output is one or two
// correctly rounded binary64 operations and is bit-reproducible.
#include "fc_kernels.hpp"

#pragma clang fp contract(off)

namespace fc {

namespace {

__global__ __launch_bounds__(256) void sum_u32_kernel(const uint32_t *__restrict__ x, int32_t n,
                                                      unsigned long long *sum) {
    unsigned long long acc = 0;
    for (int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x); i < n;
         i += static_cast<int32_t>(gridDim.x * blockDim.x))
        acc += x[i];
    // wave reduction (wave64), then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(sum, acc);
}

__global__ __launch_bounds__(256) void estimate_kernel(const uint32_t *__restrict__ R, int32_t n,
                                                       uint32_t tau, int literal,
                                                       const unsigned long long *__restrict__ sum,
                                                       double *__restrict__ diag,
                                                       double *__restrict__ farness,
                                                       double *__restrict__ closeness) {
    const int32_t v = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (v >= n) return;
    const double dt = static_cast<double>(tau);
    const uint32_t r = R[v];
    if (diag) {
        double d = static_cast<double>(r) / dt;
        if (literal) {
            // minimum-norm solution of L* x = e_{u*} - 1/(n+1) 1 gives
            // - x(u*) + 2 x(v) = -(n+2)/(n+1)^2
            const double n1 = static_cast<double>(static_cast<int64_t>(n) + 1);
            const double shift = static_cast<double>(static_cast<int64_t>(n) + 2) / (n1 * n1);
            d = d - shift;
        }
        diag[v] = d;
    }
    if (farness || closeness) {
        const unsigned long long num =
            static_cast<unsigned long long>(n) * r + *sum;
        const double f = static_cast<double>(num) / dt - 2.0;
        if (farness) farness[v] = f;
        if (closeness) closeness[v] = static_cast<double>(n) / f;
    }
}

// Plain fills (used instead of memset nodes inside captured HIP graphs).
__global__ void fill_u64_kernel(unsigned long long *__restrict__ p, size_t count,
                                unsigned long long value) {
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = value;
}

}  // namespace

hipError_t launch_fill_u64(unsigned long long *p, size_t count, unsigned long long value,
                           hipStream_t stream) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    fill_u64_kernel<<<static_cast<unsigned int>(blocks), 256, 0, stream>>>(p, count, value);
    return hipGetLastError();
}

hipError_t launch_sum_u32(const uint32_t *x, int32_t n, unsigned long long *sum,
                          hipStream_t stream) {
    if (n == 0) return hipSuccess;
    int blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    sum_u32_kernel<<<blocks, 256, 0, stream>>>(x, n, sum);
    return hipGetLastError();
}

hipError_t launch_estimate(const uint32_t *R, int32_t n, uint32_t tau, int literal,
                           const unsigned long long *sum, double *diag, double *farness,
                           double *closeness, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    estimate_kernel<<<(n + 255) / 256, 256, 0, stream>>>(R, n, tau, literal, sum, diag, farness,
                                                         closeness);
    return hipGetLastError();
}

}  // namespace fc
