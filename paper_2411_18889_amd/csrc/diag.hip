// FP64 diagnostics: kinetic, potential and total energy, linear and angular
// momentum, centre of mass and total mass of a state.
//
// The potential energy PE = -G sum_{i<j} m_i m_j / sqrt(|r_j - r_i|^2 + eps^2)
// is evaluated as -G/2 sum_i m_i (phi_i - m_i / eps), where phi_i is the
// FP64 sum over all j of m_j / sqrt(...) from the pair kernel (j = i
// included, then removed). The per-particle terms are reduced in a fixed
// order (fixed grid, fixed tree), so the result is bitwise reproducible.
#include "common.h"

namespace nb {

namespace {

constexpr int TPB = 256;
constexpr int NV = 13;  // output slots; slot 2 (E) is formed at the end

inline int diag_blocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    return (int)(b > 1024 ? 1024 : b);
}

template <typename T>
__device__ __forceinline__ void block_sum(T (&v)[NV], T* lds) {
    // one quantity at a time through a TPB-wide LDS tree
    for (int q = 0; q < NV; ++q) {
        lds[threadIdx.x] = v[q];
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
            __syncthreads();
        }
        v[q] = lds[0];
        __syncthreads();
    }
}

template <typename P, typename M>
__global__ __launch_bounds__(TPB) void diag_blocks_kernel(const P* __restrict__ x, const P* __restrict__ v,
                                                          const M* __restrict__ m,
                                                          const double* __restrict__ part, int nsplit,
                                                          int64_t n, double inv_eps,
                                                          double* __restrict__ blocks) {
    __shared__ double lds[TPB];
    double acc[NV];
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const double mi = double(m[i]);
        const double rx = double(x[i]), ry = double(x[n + i]), rz = double(x[2 * n + i]);
        const double vx = double(v[i]), vy = double(v[n + i]), vz = double(v[2 * n + i]);
        double phi = 0.0;
        for (int s = 0; s < nsplit; ++s) phi += part[((size_t)s * 4 + 3) * n + i];
        acc[0] += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
        acc[1] += mi * (phi - mi * inv_eps);
        acc[3] += mi * vx;
        acc[4] += mi * vy;
        acc[5] += mi * vz;
        acc[6] += mi * (ry * vz - rz * vy);
        acc[7] += mi * (rz * vx - rx * vz);
        acc[8] += mi * (rx * vy - ry * vx);
        acc[9] += mi * rx;
        acc[10] += mi * ry;
        acc[11] += mi * rz;
        acc[12] += mi;
    }
    block_sum(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) blocks[(size_t)blockIdx.x * NV + q] = acc[q];
}

__global__ __launch_bounds__(TPB) void diag_final_kernel(const double* __restrict__ blocks, int nblocks,
                                                         double G, double* __restrict__ out) {
    __shared__ double lds[TPB];
    double acc[NV];
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += TPB)
        for (int q = 0; q < NV; ++q) acc[q] += blocks[(size_t)b * NV + q];
    block_sum(acc, lds);
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = -0.5 * G * acc[1];
        out[2] = out[0] + out[1];
        for (int q = 3; q < 9; ++q) out[q] = acc[q];
        out[9] = acc[9] / acc[12];
        out[10] = acc[10] / acc[12];
        out[11] = acc[11] / acc[12];
        out[12] = acc[12];
    }
}

}  // namespace

size_t diag_workspace_bytes(int64_t n) {
    size_t pot = potential_partials_bytes(n);
    pot = (pot + 255) / 256 * 256;
    return pot + (size_t)diag_blocks(n) * NV * sizeof(double);
}

hipError_t launch_diag(int prec, int64_t n, const void* x, const void* v, const void* m, double eps,
                       double G, double* out, void* ws, hipStream_t stream) {
    double* part = static_cast<double*>(ws);
    size_t pot = (potential_partials_bytes(n) + 255) / 256 * 256;
    double* blocks = reinterpret_cast<double*>(static_cast<char*>(ws) + pot);
    int nsplit = 0;
    hipError_t e = launch_potential_partials(prec, n, x, m, eps, part, &nsplit, stream);
    if (e != hipSuccess) return e;
    const int nb = diag_blocks(n);
    // the j = i term of the pair sum is m_i / eps with eps as the pair kernel saw it
    const double inv_eps = 1.0 / eps;
    if (prec == NB_F32)
        hipLaunchKernelGGL((diag_blocks_kernel<float, float>), dim3(nb), dim3(TPB), 0, stream,
                           static_cast<const float*>(x), static_cast<const float*>(v),
                           static_cast<const float*>(m), part, nsplit, n, inv_eps, blocks);
    else if (prec == NB_F64)
        hipLaunchKernelGGL((diag_blocks_kernel<double, double>), dim3(nb), dim3(TPB), 0, stream,
                           static_cast<const double*>(x), static_cast<const double*>(v),
                           static_cast<const double*>(m), part, nsplit, n, inv_eps, blocks);
    else
        hipLaunchKernelGGL((diag_blocks_kernel<double, float>), dim3(nb), dim3(TPB), 0, stream,
                           static_cast<const double*>(x), static_cast<const double*>(v),
                           static_cast<const float*>(m), part, nsplit, n, inv_eps, blocks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(TPB), 0, stream, blocks, nb, G, out);
    return hipGetLastError();
}

}  // namespace nb
