// Fused adjoint pair kernel for the reverse KDK walk on gfx950.
//
// For sinks k at positions x (all particles are both sinks and sources) and
// an adjoint vector lam (the velocity adjoint), one pass over all pairs
// computes, with d = r_j - r_k, s = |d|^2 + eps^2, T(d) = s^-3/2 I
// - 3 s^-5/2 d d^T (the derivative of d s^-3/2, symmetric and even in d):
//   a_k        = G sum_j m_j d s^-3/2                      (Eq. (1))
//   (J^T lam)_k = G sum_j T(d) (m_k lam_j - m_j lam_k)      (position adjoint)
//   (G^T lam)_k = -G sum_j (lam_j . d) s^-3/2               (mass adjoint)
// The j = k term is zero in all three (d = 0 and m_k lam_k - m_k lam_k = 0).
// The first is needed to walk the state back one step and comes almost
// free: it shares d, s and the reciprocal square root. A pass that does not
// walk the state back (the entry pass, a state reloaded from a checkpoint)
// leaves it out: 6 % (FP64) to 20 % (mixed, FP64 sums) faster at 262144.
//
// Per pair, with u = m_k lam_j - m_j lam_k and e = -3 s^-1 (d . u):
//   T(d) u = s^-3/2 (u + e d)
// i.e. 6 operations for u, 3 for d.u, 2 for e, 3 FMAs for u + e d and 3 for
// the sum; plus 4 for the mass adjoint and the 12 + rsqrt of the force:
// 34 VALU + 1 rsqrt.
//
// Tiling, j-split, the origin of the pair arithmetic in the mixed policies
// and the fixed-order split reduction are as in the force kernel; the LDS record of a source is (x, y, z, m) and (lam_x, lam_y,
// lam_z, 0).
#include <algorithm>

#include "common.h"

namespace nb {

namespace {

constexpr int NQ = 7;  // partials per sink: a (3), J^T lam (3), G^T lam (1)

template <class Pol>
struct AdjArgs {
    using pos_t = typename Pol::pos_t;
    using mass_t = typename Pol::mass_t;
    using calc_t = typename Pol::calc_t;
    const pos_t *x, *y, *z;
    const mass_t* m;
    const pos_t *lx, *ly, *lz;  // lam_v (read only)
    int n;
    int jspan;
    calc_t eps2;
    double G;
    double c;      // weight of the position / mass adjoint update
    double h;      // half step, for the velocity walk-back
    int update_state;
    pos_t *ax, *ay, *az;   // acceleration out (update_state)
    pos_t *vx, *vy, *vz;   // velocity in/out (update_state)
    pos_t *gx, *gy, *gz;   // lam_x in/out
    double* gm;            // lam_m in/out
    pos_t *rx, *ry, *rz;   // x of the next step's reverse drift, or nullptr
    pos_t *rlx, *rly, *rlz;  // lam_v written by that drift
    double dt;
    double* part;          // [nsplit][NQ][n] or nullptr
};

template <class Pol>
__device__ __forceinline__ void finish_adj(const AdjArgs<Pol>& a, int i, const double q[NQ]) {
    using pos_t = typename Pol::pos_t;
    const double G = a.G, c = a.c;
    a.gx[i] = pos_t(double(a.gx[i]) + c * (G * q[3]));
    a.gy[i] = pos_t(double(a.gy[i]) + c * (G * q[4]));
    a.gz[i] = pos_t(double(a.gz[i]) + c * (G * q[5]));
    a.gm[i] = a.gm[i] + c * (-G * q[6]);
    if (a.update_state) {
        const pos_t ax = pos_t(G * q[0]), ay = pos_t(G * q[1]), az = pos_t(G * q[2]);
        const pos_t h = pos_t(a.h);
        a.ax[i] = ax;
        a.ay[i] = ay;
        a.az[i] = az;
        a.vx[i] = fmat(-h, ax, a.vx[i]);
        a.vy[i] = fmat(-h, ay, a.vy[i]);
        a.vz[i] = fmat(-h, az, a.vz[i]);
    }
    if (a.rx) {  // the next step's reverse drift, as the reverse-drift kernel does it
        const pos_t h = pos_t(a.h), dt = pos_t(a.dt);
        a.rlx[i] = fmat(dt, a.gx[i], a.rlx[i]);
        a.rly[i] = fmat(dt, a.gy[i], a.rly[i]);
        a.rlz[i] = fmat(dt, a.gz[i], a.rlz[i]);
        const pos_t vx = fmat(-h, a.ax[i], a.vx[i]), vy = fmat(-h, a.ay[i], a.vy[i]),
                    vz = fmat(-h, a.az[i], a.vz[i]);
        a.vx[i] = vx;
        a.vy[i] = vy;
        a.vz[i] = vz;
        a.rx[i] = fmat(-dt, vx, a.rx[i]);
        a.ry[i] = fmat(-dt, vy, a.ry[i]);
        a.rz[i] = fmat(-dt, vz, a.rz[i]);
    }
}

// F: also sum the force a (quantities 0..2, for a pass that walks the state
// back); without it they stay 0 and the pair body is 4 operations shorter.
template <class Pol, int BS, int K, bool F>
__global__ __launch_bounds__(BS) void adjoint_kernel(AdjArgs<Pol> a) {
    using calc_t = typename Pol::calc_t;
    using sum_t = typename Pol::sum_t;
    using V4 = typename Vec4<calc_t>::type;
    __shared__ V4 tp[BS];
    __shared__ V4 tl[BS];

    const int tid = threadIdx.x;
    const int b0 = blockIdx.x * (BS * K);
    const int i0 = b0 + tid;
    // origin of the pair arithmetic (mixed policies): the centroid of this
    // workgroup's sinks
    double ox = 0.0, oy = 0.0, oz = 0.0;
    if constexpr (Pol::origin) {
        __shared__ double org[BS / 64][3];
        double cx = 0.0, cy = 0.0, cz = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + k * BS;
            if (i < a.n) {
                cx += a.x[i];
                cy += a.y[i];
                cz += a.z[i];
            }
        }
        sink_block_origin<BS / 64>(cx, cy, cz, min(a.n - b0, BS * K), org, ox, oy, oz);
    }
    calc_t xi[K], yi[K], zi[K], mi[K], lxi[K], lyi[K], lzi[K];
    sum_t s[K][NQ];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k * BS;
        const bool ok = i < a.n;
        xi[k] = ok ? pair_coord<Pol>(a.x[i], ox) : calc_t(0);
        yi[k] = ok ? pair_coord<Pol>(a.y[i], oy) : calc_t(0);
        zi[k] = ok ? pair_coord<Pol>(a.z[i], oz) : calc_t(0);
        mi[k] = ok ? calc_t(a.m[i]) : calc_t(0);
        lxi[k] = ok ? calc_t(a.lx[i]) : calc_t(0);
        lyi[k] = ok ? calc_t(a.ly[i]) : calc_t(0);
        lzi[k] = ok ? calc_t(a.lz[i]) : calc_t(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[k][q].init();
    }
    const calc_t eps2 = a.eps2;
    const int jbeg = blockIdx.y * a.jspan;
    const int jend = min(a.n, jbeg + a.jspan);

    for (int jt = jbeg; jt < jend; jt += BS) {
        const int j = jt + tid;
        V4 p, l;
        if (j < jend) {
            p.x = pair_coord<Pol>(a.x[j], ox);
            p.y = pair_coord<Pol>(a.y[j], oy);
            p.z = pair_coord<Pol>(a.z[j], oz);
            p.w = calc_t(a.m[j]);
            l.x = calc_t(a.lx[j]); l.y = calc_t(a.ly[j]); l.z = calc_t(a.lz[j]); l.w = calc_t(0);
        } else {  // zero mass and zero adjoint: contributes exactly 0
            p.x = p.y = p.z = p.w = calc_t(0);
            l.x = l.y = l.z = l.w = calc_t(0);
        }
        __syncthreads();
        tp[tid] = p;
        tl[tid] = l;
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < BS; ++jj) {
            const V4 q = tp[jj];
            const V4 lj = tl[jj];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const calc_t dx = q.x - xi[k];
                const calc_t dy = q.y - yi[k];
                const calc_t dz = q.z - zi[k];
                const calc_t ss = fmat(dz, dz, fmat(dy, dy, fmat(dx, dx, eps2)));
                const calc_t r = rsqrt_pair(ss);
                const calc_t r2 = r * r;
                const calc_t r3 = r2 * r;
                if (F) {  // force
                    const calc_t w = r3 * q.w;
                    s[k][0].add_fma(dx, w);
                    s[k][1].add_fma(dy, w);
                    s[k][2].add_fma(dz, w);
                }
                // position adjoint: T(d) u = r3 (u + e d), e = -3 r2 (d . u)
                const calc_t ux = fmat(mi[k], lj.x, -(q.w * lxi[k]));
                const calc_t uy = fmat(mi[k], lj.y, -(q.w * lyi[k]));
                const calc_t uz = fmat(mi[k], lj.z, -(q.w * lzi[k]));
                const calc_t du = fmat(dz, uz, fmat(dy, uy, dx * ux));
                const calc_t e = (calc_t(-3) * r2) * du;
                s[k][3].add_fma(r3, fmat(e, dx, ux));
                s[k][4].add_fma(r3, fmat(e, dy, uy));
                s[k][5].add_fma(r3, fmat(e, dz, uz));
                // mass adjoint (sign applied at the end)
                const calc_t dl = fmat(dz, lj.z, fmat(dy, lj.y, dx * lj.x));
                s[k][6].add_fma(r3, dl);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < NQ; ++q) s[k][q].tile_end();
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k * BS;
        if (i >= a.n) continue;
        if (a.part) {
            double* out = a.part + (size_t)blockIdx.y * NQ * a.n;
#pragma unroll
            for (int q = 0; q < NQ; ++q) out[(size_t)q * a.n + i] = s[k][q].total();
        } else {
            double t[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) t[q] = s[k][q].total();
            finish_adj<Pol>(a, i, t);
        }
    }
}

template <class Pol>
__global__ __launch_bounds__(256) void adjoint_reduce_kernel(AdjArgs<Pol> a, int nsplit) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    double t[NQ] = {0, 0, 0, 0, 0, 0, 0};
    // four ranges' loads in flight together, the adds in range order
#pragma unroll 4
    for (int sp = 0; sp < nsplit; ++sp) {
        const double* q = a.part + (size_t)sp * NQ * a.n;
#pragma unroll
        for (int c = 0; c < NQ; ++c) t[c] += q[(size_t)c * a.n + i];
    }
    finish_adj<Pol>(a, i, t);
}

int split_span(int64_t n, int split, int block) {
    int64_t per = (n + split - 1) / split;
    per = (per + block - 1) / block * block;
    return (int)per;
}

template <class Pol, int BS, int K>
hipError_t launch_shape(AdjArgs<Pol> a, int nsplit, hipStream_t stream) {
    dim3 grid((a.n + BS * K - 1) / (BS * K), nsplit);
    if (a.update_state)
        hipLaunchKernelGGL((adjoint_kernel<Pol, BS, K, true>), grid, dim3(BS), 0, stream, a);
    else
        hipLaunchKernelGGL((adjoint_kernel<Pol, BS, K, false>), grid, dim3(BS), 0, stream, a);
    return hipGetLastError();
}

template <class Pol>
hipError_t launch_any(const Shape& sh, AdjArgs<Pol> a, int nsplit, hipStream_t stream) {
#define NB_ADJ_CASE(BSV, KV) \
    if (sh.block == BSV && sh.ipl == KV) return launch_shape<Pol, BSV, KV>(a, nsplit, stream);
    NB_ADJ_CASE(64, 1) NB_ADJ_CASE(64, 2)
    NB_ADJ_CASE(128, 1) NB_ADJ_CASE(128, 2)
    NB_ADJ_CASE(256, 1) NB_ADJ_CASE(256, 2)
    NB_ADJ_CASE(512, 1) NB_ADJ_CASE(512, 2)
#undef NB_ADJ_CASE
    return hipErrorInvalidValue;
}

}  // namespace

Shape choose_adjoint_shape(int prec, int64_t n) {
    // Measured on MI355X: one sink per lane (the fused pair body is long
    // enough to hide latency on its own; two sinks per lane run 13 % slower),
    // 512-lane workgroups from 2^19 sinks up, 256 from 4096, 64 below; a
    // source split up to ~128K wavefronts (8 ranges at 2^20), every range
    // >= 2 tiles long (4 below 32768 sinks) -- or, below 16384 sinks, as
    // short as one tile up to 32 ranges (2.2-2.8x faster at N = 1024 and
    // 2048, where the pass is otherwise a handful of workgroups).
    (void)prec;
    Shape s{1, n >= (1 << 19) ? 512 : (n <= 2048 ? 64 : 256), 1};
    const int64_t waves = (n + s.block - 1) / s.block * (s.block / 64);
    const int64_t want = 131072;
    int64_t split = (want + waves - 1) / waves;
    const int64_t long_ranges = n / ((n < 32768 ? 4 : 2) * (int64_t)s.block);
    const int64_t short_ranges = n < 16384 ? std::min<int64_t>(32, n / (int64_t)s.block) : 0;
    const int64_t max_ranges = std::max(long_ranges, short_ranges);
    if (split > max_ranges) split = max_ranges;
    if (split > 256) split = 256;
    if (split < 1) split = 1;
    s.split = (int)split;
    return s;
}

bool adjoint_shape_supported(const Shape& s) {
    const bool bs_ok = s.block == 64 || s.block == 128 || s.block == 256 || s.block == 512;
    return bs_ok && (s.ipl == 1 || s.ipl == 2) && s.split >= 1 && s.split <= 256;
}

size_t adjoint_partials_bytes(const Shape& s, int64_t n) {
    return (size_t)s.split * NQ * (size_t)n * sizeof(double);
}

hipError_t launch_adjoint(int prec, const Shape& sh, int64_t n, const void* x, const void* m,
                          const void* lam_v, double eps, double G, double c, bool update_state,
                          double h, void* acc, void* v, void* lam_x, double* lam_m, void* ws,
                          hipStream_t stream, void* drift_x, double drift_dt, bool* drifted) {
    hipError_t err = hipErrorInvalidValue;
    if (drifted) *drifted = false;
    dispatch_prec(prec, [&](auto tag) {
        using Pol = decltype(tag);
        using pos_t = typename Pol::pos_t;
        using mass_t = typename Pol::mass_t;
        using calc_t = typename Pol::calc_t;
        AdjArgs<Pol> a{};
        const pos_t* px = static_cast<const pos_t*>(x);
        const pos_t* pl = static_cast<const pos_t*>(lam_v);
        a.x = px; a.y = px + n; a.z = px + 2 * n;
        a.m = static_cast<const mass_t*>(m);
        a.lx = pl; a.ly = pl + n; a.lz = pl + 2 * n;
        a.n = (int)n;
        a.eps2 = calc_t(eps) * calc_t(eps);
        a.G = G;
        a.c = c;
        a.h = h;
        a.update_state = update_state ? 1 : 0;
        pos_t* pa = static_cast<pos_t*>(acc);
        pos_t* pv = static_cast<pos_t*>(v);
        pos_t* pg = static_cast<pos_t*>(lam_x);
        a.ax = pa; a.ay = pa + n; a.az = pa + 2 * n;
        a.vx = pv; a.vy = pv + n; a.vz = pv + 2 * n;
        a.gx = pg; a.gy = pg + n; a.gz = pg + 2 * n;
        a.gm = lam_m;
        const int span = split_span(n, sh.split, sh.block);
        const int nsplit = (int)((n + span - 1) / span);
        a.jspan = span;
        if (nsplit == 1) {  // sinks finish while others still read x and lam_v: no drift
            a.part = nullptr;
            err = launch_any<Pol>(sh, a, 1, stream);
            return;
        }
        if (drift_x) {
            pos_t* prx = static_cast<pos_t*>(drift_x);
            pos_t* prl = static_cast<pos_t*>(const_cast<void*>(lam_v));
            a.rx = prx; a.ry = prx + n; a.rz = prx + 2 * n;
            a.rlx = prl; a.rly = prl + n; a.rlz = prl + 2 * n;
            a.dt = drift_dt;
            if (drifted) *drifted = true;
        }
        a.part = static_cast<double*>(ws);
        err = launch_any<Pol>(sh, a, nsplit, stream);
        if (err != hipSuccess) return;
        hipLaunchKernelGGL((adjoint_reduce_kernel<Pol>), dim3((a.n + 255) / 256), dim3(256), 0,
                           stream, a, nsplit);
        err = hipGetLastError();
    });
    return err;
}

}  // namespace nb
