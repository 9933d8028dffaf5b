// FP64 diagnostics: kinetic, potential and total energy, linear and angular
// momentum, centre of mass and total mass of a state.
//
// Potential energy PE = -G sum_{i<j} m_i m_j / sqrt(|r_j - r_i|^2 + eps^2):
// only the pairs i < j are visited. The particles are cut into tiles of
// PT = 1024; the tile pairs (I, J) with I <= J are enumerated linearly and
// dealt round-robin to a fixed grid of workgroups; a workgroup holds the 1024
// sinks of tile I in registers (4 per lane) and streams tile J through LDS.
// Diagonal tile pairs keep j > i only. Every workgroup adds its pairs into
// one FP64 partial; the partials and the per-particle terms of KE, P, L and
// the centre of mass are reduced in a fixed order (fixed grid, fixed trees),
// so the result is bitwise reproducible.
//
// Reciprocal square root: v_rsq_f64 (about 24 correct bits) and one
// Newton-Raphson step, which leaves a relative error of a few 1e-15 per term.
#include "common.h"

namespace nb {

namespace {

constexpr int TPB = 256;
constexpr int PT = 1024;            // particles per potential tile
constexpr int PK = PT / TPB;        // sinks per lane
constexpr int PE_GRID = 16384;      // workgroups of the potential pass
constexpr int NV = 13;              // output slots; slot 1 (PE) and 2 (E) formed at the end

inline int diag_blocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    return (int)(b > 1024 ? 1024 : b);
}

__device__ __forceinline__ double rsqrt_1nr(double s) {
    double y = __builtin_amdgcn_rsq(s);
    const double e = __builtin_fma(-s * y, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double* lds) {
    for (int q = 0; q < NQ; ++q) {
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

// Workgroup b visits tile pairs t = b, b + PE_GRID, ... < ntiles (ntiles + 1) / 2.
template <typename P, typename M>
__global__ __launch_bounds__(TPB) void pe_pairs_kernel(const P* __restrict__ x, const M* __restrict__ m,
                                                       int64_t n, double eps2, int64_t ntiles,
                                                       double* __restrict__ part) {
    __shared__ double4 tile[PT];
    __shared__ double lds[TPB];
    const P* y = x + n;
    const P* z = x + 2 * n;
    const int64_t npairs = ntiles * (ntiles + 1) / 2;
    double total = 0.0;
    for (int64_t t = blockIdx.x; t < npairs; t += gridDim.x) {
        // t -> (I, J), I <= J, with t = J (J + 1) / 2 + I
        int64_t J = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (J * (J + 1) / 2 > t) --J;
        while ((J + 1) * (J + 2) / 2 <= t) ++J;
        const int64_t I = t - J * (J + 1) / 2;
        double xi[PK], yi[PK], zi[PK], acc[PK];
        int64_t iidx[PK];
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int64_t i = I * PT + k * TPB + threadIdx.x;
            iidx[k] = i;
            const bool ok = i < n;
            xi[k] = ok ? double(x[i]) : 0.0;
            yi[k] = ok ? double(y[i]) : 0.0;
            zi[k] = ok ? double(z[i]) : 0.0;
            acc[k] = 0.0;
        }
        __syncthreads();  // previous tile fully consumed
        for (int q = threadIdx.x; q < PT; q += TPB) {
            const int64_t j = J * PT + q;
            double4 r;
            if (j < n) {
                r.x = double(x[j]); r.y = double(y[j]); r.z = double(z[j]); r.w = double(m[j]);
            } else {
                r.x = r.y = r.z = r.w = 0.0;  // zero mass: adds exactly 0
            }
            tile[q] = r;
        }
        __syncthreads();
        if (I != J) {
            for (int q = 0; q < PT; ++q) {
                const double4 r = tile[q];
#pragma unroll
                for (int k = 0; k < PK; ++k) {
                    const double dx = r.x - xi[k], dy = r.y - yi[k], dz = r.z - zi[k];
                    const double s = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
                    acc[k] = __builtin_fma(r.w, rsqrt_1nr(s), acc[k]);
                }
            }
        } else {  // same tile: only j > i
            for (int q = 0; q < PT; ++q) {
                const double4 r = tile[q];
                const int64_t j = J * PT + q;
#pragma unroll
                for (int k = 0; k < PK; ++k) {
                    const double dx = r.x - xi[k], dy = r.y - yi[k], dz = r.z - zi[k];
                    const double s = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, eps2)));
                    const double term = r.w * rsqrt_1nr(s);
                    acc[k] += (j > iidx[k]) ? term : 0.0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < PK; ++k)
            if (iidx[k] < n) total = __builtin_fma(double(m[iidx[k]]), acc[k], total);
    }
    double v[1] = {total};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename P, typename M>
__global__ __launch_bounds__(TPB) void diag_blocks_kernel(const P* __restrict__ x, const P* __restrict__ v,
                                                          const M* __restrict__ m, int64_t n,
                                                          double* __restrict__ blocks) {
    __shared__ double lds[TPB];
    double acc[NV];
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
        const double mi = double(m[i]);
        const double rx = double(x[i]), ry = double(x[n + i]), rz = double(x[2 * n + i]);
        const double vx = double(v[i]), vy = double(v[n + i]), vz = double(v[2 * n + i]);
        acc[0] += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
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
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) blocks[(size_t)blockIdx.x * NV + q] = acc[q];
}

__global__ __launch_bounds__(TPB) void diag_final_kernel(const double* __restrict__ blocks, int nblocks,
                                                         const double* __restrict__ pe_part, int npe,
                                                         double G, double* __restrict__ out) {
    __shared__ double lds[TPB];
    double acc[NV];
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += TPB)
        for (int q = 0; q < NV; ++q) acc[q] += blocks[(size_t)b * NV + q];
    for (int b = threadIdx.x; b < npe; b += TPB) acc[1] += pe_part[b];
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = -G * acc[1];
        out[2] = out[0] + out[1];
        for (int q = 3; q < 9; ++q) out[q] = acc[q];
        out[9] = acc[9] / acc[12];
        out[10] = acc[10] / acc[12];
        out[11] = acc[11] / acc[12];
        out[12] = acc[12];
    }
}

template <typename P, typename M>
hipError_t run_diag(int64_t n, const void* x, const void* v, const void* m, double eps, double G,
                    double* out, void* ws, hipStream_t stream) {
    double* pe_part = static_cast<double*>(ws);
    double* blocks = pe_part + PE_GRID;
    const int64_t ntiles = (n + PT - 1) / PT;
    const int64_t npairs = ntiles * (ntiles + 1) / 2;
    const int grid = (int)(npairs < PE_GRID ? npairs : PE_GRID);
    hipLaunchKernelGGL((pe_pairs_kernel<P, M>), dim3(grid), dim3(TPB), 0, stream,
                       static_cast<const P*>(x), static_cast<const M*>(m), n, eps * eps, ntiles, pe_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb = diag_blocks(n);
    hipLaunchKernelGGL((diag_blocks_kernel<P, M>), dim3(nb), dim3(TPB), 0, stream, static_cast<const P*>(x),
                       static_cast<const P*>(v), static_cast<const M*>(m), n, blocks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(TPB), 0, stream, blocks, nb, pe_part, grid, G, out);
    return hipGetLastError();
}

}  // namespace

size_t diag_workspace_bytes(int64_t n) {
    return ((size_t)PE_GRID + (size_t)diag_blocks(n) * NV) * sizeof(double);
}

hipError_t launch_diag(int prec, int64_t n, const void* x, const void* v, const void* m, double eps,
                       double G, double* out, void* ws, hipStream_t stream) {
    if (prec == NB_F32) return run_diag<float, float>(n, x, v, m, eps, G, out, ws, stream);
    if (prec == NB_F64) return run_diag<double, double>(n, x, v, m, eps, G, out, ws, stream);
    return run_diag<double, float>(n, x, v, m, eps, G, out, ws, stream);
}

}  // namespace nb
