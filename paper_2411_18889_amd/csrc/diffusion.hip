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

// Vector form for nz % 4 == 0: every lane owns 4 consecutive k points
// (16-byte loads and stores), a wave covers 256 k points of one row, a
// workgroup TJ4 rows; the plane two steps ahead is already in flight while
// the current one is computed, so each wave keeps 2 KB of loads outstanding.
// The j +- 1 rows go through LDS (row layout [.., 256 points at V_OFF..] with
// V_OFF = 4 so each lane's 4 points are a 16-byte access); the k +- 1
// neighbours of a lane's 4 points are the adjacent lanes' end points, taken
// with DPP wave shifts -- reading them from LDS at a 4-float stride cost
// 4-way bank conflicts (a third of the LDS cycles) and 6-9 % at 512^3.
constexpr int TK4 = 256;
constexpr int TJ4 = 16;
constexpr int CI4 = 64;
constexpr int V_OFF = 4;
constexpr int ROW = TK4 + 2 * V_OFF;

__device__ __forceinline__ float4 load_row4(const float* __restrict__ f, int64_t row, int k0, int nz) {
    // the 4 points k0..k0+3 of a row; lanes past the end of the row take the
    // row's last point in every slot, which is what the clamped neighbour rule
    // asks of the point before them
    if (k0 < nz) return *reinterpret_cast<const float4*>(f + row + k0);
    const float e = f[row + nz - 1];
    return make_float4(e, e, e, e);
}

__global__ __launch_bounds__(64 * TJ4) void diffusion_kernel4(int nx, int ny, int nz, Coef c,
                                                              const float* __restrict__ f,
                                                              float* __restrict__ fn) {
    __shared__ __align__(16) float pl[TJ4 + 2][ROW];
    const int lane = threadIdx.x, ty = threadIdx.y;
    const int k0 = blockIdx.x * TK4 + 4 * lane;
    const int j = blockIdx.y * TJ4 + ty;
    const int jc = min(j, ny - 1);
    const int i0 = blockIdx.z * CI4, i1 = min(i0 + CI4, nx);
    const int64_t plane = (int64_t)ny * nz;
    const int64_t row = (int64_t)jc * nz;
    const int64_t row_jm = (int64_t)max(j - 1, 0) * nz;
    const int64_t row_jp = (int64_t)min(j + 1, ny - 1) * nz;
    const int kl = blockIdx.x * TK4 - 1, kr = blockIdx.x * TK4 + TK4;  // tile halo points
    const bool store = k0 < nz && j < ny;

    float4 prev = load_row4(f, (int64_t)max(i0 - 1, 0) * plane + row, k0, nz);
    float4 cur = load_row4(f, (int64_t)i0 * plane + row, k0, nz);
    float4 next = load_row4(f, (int64_t)min(i0 + 1, nx - 1) * plane + row, k0, nz);
    for (int i = i0; i < i1; ++i) {
        const int64_t base = (int64_t)i * plane;
        const float4 after = load_row4(f, (int64_t)min(i + 2, nx - 1) * plane + row, k0, nz);
        __syncthreads();  // the previous plane has been read by every lane
        *reinterpret_cast<float4*>(&pl[ty + 1][V_OFF + 4 * lane]) = cur;
        // k neighbours across lanes come from the adjacent lanes (DPP wave
        // shifts); the tile's two halo points, needed by lanes 0 and 63 only,
        // are read by the whole wave from one address each
        const float hl = f[base + row + max(kl, 0)];
        const float hr = f[base + row + min(kr, nz - 1)];
        if (ty == 0) {
            *reinterpret_cast<float4*>(&pl[0][V_OFF + 4 * lane]) = load_row4(f, base + row_jm, k0, nz);
        }
        if (ty == TJ4 - 1) {
            *reinterpret_cast<float4*>(&pl[TJ4 + 1][V_OFF + 4 * lane]) = load_row4(f, base + row_jp, k0, nz);
        }
        __syncthreads();
        if (store) {
            const float4 jp = *reinterpret_cast<const float4*>(&pl[ty + 2][V_OFF + 4 * lane]);
            const float4 jm = *reinterpret_cast<const float4*>(&pl[ty][V_OFF + 4 * lane]);
            const float km0 = __int_as_float(__builtin_amdgcn_update_dpp(
                __float_as_int(hl), __float_as_int(cur.w), 0x138, 0xF, 0xF, false));  // lane - 1
            const float kp3 = __int_as_float(__builtin_amdgcn_update_dpp(
                __float_as_int(hr), __float_as_int(cur.x), 0x130, 0xF, 0xF, false));  // lane + 1
            // the last point of the grid has itself as its k+1 neighbour
            const float kp3c = (k0 + 4 < nz) ? kp3 : cur.w;
            const float km0c = (k0 > 0) ? km0 : cur.x;
            float4 r;
#define NB_DIFF_POINT(OUT, C, N, P, JP, JM, KP, KM)                 \
    {                                                               \
        float t = c.cc * (C);                                       \
        t = __builtin_fmaf(c.ce, (N), t);                           \
        t = __builtin_fmaf(c.cw, (P), t);                           \
        t = __builtin_fmaf(c.cn, (JP), t);                          \
        t = __builtin_fmaf(c.cs, (JM), t);                          \
        t = __builtin_fmaf(c.ct, (KP), t);                          \
        OUT = __builtin_fmaf(c.cb, (KM), t);                        \
    }
            NB_DIFF_POINT(r.x, cur.x, next.x, prev.x, jp.x, jm.x, cur.y, km0c)
            NB_DIFF_POINT(r.y, cur.y, next.y, prev.y, jp.y, jm.y, cur.z, cur.x)
            NB_DIFF_POINT(r.z, cur.z, next.z, prev.z, jp.z, jm.z, cur.w, cur.y)
            NB_DIFF_POINT(r.w, cur.w, next.w, prev.w, jp.w, jm.w, kp3c, cur.z)
#undef NB_DIFF_POINT
            // streaming store: fn is not read again by this step
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f rv = {r.x, r.y, r.z, r.w};
            __builtin_nontemporal_store(rv, reinterpret_cast<v4f*>(fn + base + row + k0));
        }
        prev = cur;
        cur = next;
        next = after;
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
    const bool vec = nz % 4 == 0 && reinterpret_cast<uintptr_t>(f) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(fn) % 16 == 0 && (ny + TJ4 - 1) / TJ4 <= 65535;
    if (vec) {
        const dim3 grid4((unsigned)((nz + TK4 - 1) / TK4), (unsigned)((ny + TJ4 - 1) / TJ4),
                         (unsigned)((nx + CI4 - 1) / CI4));
        hipLaunchKernelGGL(diffusion_kernel4, grid4, dim3(64, TJ4), 0, stream, (int)nx, (int)ny, (int)nz,
                           c, f, fn);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((nz + TK - 1) / TK), (unsigned)((ny + TJ - 1) / TJ),
                    (unsigned)((nx + CI - 1) / CI));
    hipLaunchKernelGGL(diffusion_kernel, grid, dim3(TK, TJ), 0, stream, (int)nx, (int)ny, (int)nz, c, f,
                       fn);
    return hipGetLastError();
}

}  // namespace nb
