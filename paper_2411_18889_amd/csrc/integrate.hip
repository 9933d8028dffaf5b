// O(N) kernels of the kick-drift-kick leapfrog and of its reverse walk (the
// closing half-kick of a step runs in the force kernel's epilogue). Each
// thread updates components of the 3n-element SoA arrays; all accesses are
// unit-stride and coalesced. These kernels are bound by HBM traffic, not
// arithmetic: per component a kick-drift moves 5 values, a reverse drift 7.
#include "common.h"

namespace nb {

namespace {

constexpr int TPB = 256;

inline dim3 grid_for(int64_t count) {
    int64_t blocks = (count + TPB - 1) / TPB;
    if (blocks > 65536) blocks = 65536;  // grid-stride beyond this
    return dim3((unsigned)blocks);
}

// v <- v + h a; x <- x + dt v
template <typename T>
__global__ __launch_bounds__(TPB) void kick_drift_kernel(T* __restrict__ x, T* __restrict__ v,
                                                         const T* __restrict__ a, T h, T dt,
                                                         int64_t count) {
    for (int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * TPB) {
        const T vh = fmat(h, a[k], v[k]);  // the same FMAs as the force epilogue's
        v[k] = vh;
        x[k] = fmat(dt, vh, x[k]);
    }
}

// Reverse of a drift and of the kick before it:
// lam_v <- lam_v + dt lam_x; v <- v - h a; x <- x - dt v.
template <typename T>
__global__ __launch_bounds__(TPB) void reverse_drift_kernel(T* __restrict__ x, T* __restrict__ v,
                                                            const T* __restrict__ a,
                                                            const T* __restrict__ lx,
                                                            T* __restrict__ lv, T h, T dt,
                                                            int64_t count) {
    for (int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * TPB) {
        lv[k] = fmat(dt, lx[k], lv[k]);  // the same FMAs as the adjoint epilogue's
        const T vh = fmat(-h, a[k], v[k]);
        v[k] = vh;
        x[k] = fmat(-dt, vh, x[k]);
    }
}

template <typename T>
__global__ __launch_bounds__(TPB) void axpy_kernel(T* __restrict__ y, const T* __restrict__ x, T a,
                                                   int64_t count) {
    for (int64_t k = blockIdx.x * (int64_t)TPB + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * TPB)
        y[k] = y[k] + a * x[k];
}

}  // namespace

hipError_t launch_kick_drift(int prec, int64_t n, void* x, void* v, const void* acc, double h,
                             double dt, hipStream_t stream) {
    const int64_t c = 3 * n;
    if (prec == NB_F32)
        hipLaunchKernelGGL(kick_drift_kernel<float>, grid_for(c), dim3(TPB), 0, stream,
                           static_cast<float*>(x), static_cast<float*>(v),
                           static_cast<const float*>(acc), float(h), float(dt), c);
    else
        hipLaunchKernelGGL(kick_drift_kernel<double>, grid_for(c), dim3(TPB), 0, stream,
                           static_cast<double*>(x), static_cast<double*>(v),
                           static_cast<const double*>(acc), h, dt, c);
    return hipGetLastError();
}

hipError_t launch_reverse_drift(int prec, int64_t n, void* x, void* v, const void* acc,
                                const void* lam_x, void* lam_v, double h, double dt,
                                hipStream_t stream) {
    const int64_t c = 3 * n;
    if (prec == NB_F32)
        hipLaunchKernelGGL(reverse_drift_kernel<float>, grid_for(c), dim3(TPB), 0, stream,
                           static_cast<float*>(x), static_cast<float*>(v),
                           static_cast<const float*>(acc), static_cast<const float*>(lam_x),
                           static_cast<float*>(lam_v), float(h), float(dt), c);
    else
        hipLaunchKernelGGL(reverse_drift_kernel<double>, grid_for(c), dim3(TPB), 0, stream,
                           static_cast<double*>(x), static_cast<double*>(v),
                           static_cast<const double*>(acc), static_cast<const double*>(lam_x),
                           static_cast<double*>(lam_v), h, dt, c);
    return hipGetLastError();
}

hipError_t launch_axpy_pos(int prec, int64_t count, void* y, const void* x, double a,
                           hipStream_t stream) {
    if (prec == NB_F32)
        hipLaunchKernelGGL(axpy_kernel<float>, grid_for(count), dim3(TPB), 0, stream,
                           static_cast<float*>(y), static_cast<const float*>(x), float(a), count);
    else
        hipLaunchKernelGGL(axpy_kernel<double>, grid_for(count), dim3(TPB), 0, stream,
                           static_cast<double*>(y), static_cast<const double*>(x), a, count);
    return hipGetLastError();
}

}  // namespace nb
