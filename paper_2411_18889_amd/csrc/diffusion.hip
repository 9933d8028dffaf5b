// One explicit step of the 3-D diffusion equation (section "3D diffusion
// equation"): every point of an nx x ny x nz FP32 grid (k fastest) becomes
//   cc f + ce f(i+1) + cw f(i-1) + cn f(j+1) + cs f(j-1) + ct f(k+1) + cb f(k-1)
// with neighbours outside the grid replaced by the nearest point inside, in
// the listing's order (left to right, contracted into one multiply and six
// FMAs).
//
// The step moves 8 bytes per point at best (one read, one write) against 13
// flops, so it is bound by HBM. A workgroup of TK x TJ lanes owns a (k, j)
// tile and marches along i over CI planes: the i-1, i, i+1 values of its
// column stay in registers, the current plane of the tile plus a one-point
// halo goes through LDS for the j and k neighbours, so every grid value is
// read from HBM about once (plus the halos, which the neighbouring tiles read
// as their own interior and mostly hit in L2). Loads along k are contiguous
// across a wave (coalesced), and every load index is clamped into the grid.
#include "common.h"

namespace nb {

namespace {

constexpr int TK = 64;  // lanes along k (one wave per row of the tile)
constexpr int TJ = 8;   // rows along j
constexpr int CI = 32;  // planes along i per workgroup

struct Coef {
    float cc, ce, cw, cn, cs, ct, cb;
};

__global__ __launch_bounds__(TK * TJ) void diffusion_kernel(int nx, int ny, int nz, Coef c,
                                                            const float* __restrict__ f,
                                                            float* __restrict__ fn) {
    __shared__ float pl[TJ + 2][TK + 2];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int k = blockIdx.x * TK + tx, j = blockIdx.y * TJ + ty;
    const int kc = min(k, nz - 1), jc = min(j, ny - 1);
    const int i0 = blockIdx.z * CI, i1 = min(i0 + CI, nx);
    const int64_t plane = (int64_t)ny * nz;
    const int64_t col = (int64_t)jc * nz + kc;
    const int64_t col_km = (int64_t)jc * nz + max(k - 1, 0);
    const int64_t col_kp = (int64_t)jc * nz + min(k + 1, nz - 1);
    const int64_t col_jm = (int64_t)max(j - 1, 0) * nz + kc;
    const int64_t col_jp = (int64_t)min(j + 1, ny - 1) * nz + kc;
    const bool store = k < nz && j < ny;

    float prev = f[(int64_t)max(i0 - 1, 0) * plane + col];
    float cur = f[(int64_t)i0 * plane + col];
    for (int i = i0; i < i1; ++i) {
        const int64_t base = (int64_t)i * plane;
        const float next = f[(int64_t)min(i + 1, nx - 1) * plane + col];
        __syncthreads();  // the previous plane has been read by every lane
        pl[ty + 1][tx + 1] = cur;
        if (tx == 0) pl[ty + 1][0] = f[base + col_km];
        if (tx == TK - 1) pl[ty + 1][TK + 1] = f[base + col_kp];
        if (ty == 0) pl[0][tx + 1] = f[base + col_jm];
        if (ty == TJ - 1) pl[TJ + 1][tx + 1] = f[base + col_jp];
        __syncthreads();
        if (store) {
            float r = c.cc * cur;
            r = __builtin_fmaf(c.ce, next, r);
            r = __builtin_fmaf(c.cw, prev, r);
            r = __builtin_fmaf(c.cn, pl[ty + 2][tx + 1], r);
            r = __builtin_fmaf(c.cs, pl[ty][tx + 1], r);
            r = __builtin_fmaf(c.ct, pl[ty + 1][tx + 2], r);
            r = __builtin_fmaf(c.cb, pl[ty + 1][tx], r);
            fn[base + col] = r;
        }
        prev = cur;
        cur = next;
    }
}

}  // namespace

hipError_t launch_diffusion3d(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                              double dt, double kappa, const float* f, float* fn, hipStream_t stream) {
    Coef c;
    const double ce = kappa * dt / (dx * dx), cn = kappa * dt / (dy * dy), ct = kappa * dt / (dz * dz);
    c.ce = c.cw = float(ce);
    c.cn = c.cs = float(cn);
    c.ct = c.cb = float(ct);
    c.cc = float(1.0 - 2.0 * (ce + cn + ct));
    const dim3 grid((unsigned)((nz + TK - 1) / TK), (unsigned)((ny + TJ - 1) / TJ),
                    (unsigned)((nx + CI - 1) / CI));
    hipLaunchKernelGGL(diffusion_kernel, grid, dim3(TK, TJ), 0, stream, (int)nx, (int)ny, (int)nz, c, f,
                       fn);
    return hipGetLastError();
}

}  // namespace nb
