// Pair-force kernels of Eq. (1) (section "N-body simulation") for gfx950.
//
// Design (one launch = ni sinks against a range of sources):
//  * a workgroup of BS threads owns BS*K sinks; each lane keeps K sinks in
//    registers (sink k of lane t is i = group*BS*K + k*BS + t, so the SoA
//    loads and stores of a wave are contiguous);
//  * the sources are streamed in j-tiles of BS particles: every lane loads
//    one source from the SoA arrays (coalesced), rounds it to the pair
//    arithmetic type (in the mixed policies relative to the centroid of the
//    workgroup's sinks, see sink_block_origin) and stores it in LDS as
//    (x, y, z, m); after a barrier
//    every lane walks the whole tile, and every LDS read is a broadcast (all
//    lanes read the same address, so no bank conflicts);
//  * per pair: 3 subtractions, 3 FMAs for |d|^2 + eps^2 (eps^2 innermost, as
//    the listing), one reciprocal square root, 3 multiplications for
//    m_j / s^(3/2), 3 FMAs into the sums; no MFMA, since nothing here is a
//    dense contraction;
//  * small N: the source range is split over gridDim.y workgroups (j-split).
//    Each writes its FP64 partial sums to the workspace and a second kernel
//    adds them in a fixed order: no atomics, bitwise reproducible;
//  * the sum over sources includes j = i, which adds exactly 0 to a_i (d = 0)
//    and m_i / eps to the potential sum; that term is removed at the end.
#include <algorithm>

#include "common.h"

namespace nb {

namespace {

constexpr int NQ = 4;  // partial quantities per sink: ax, ay, az, potential

template <class Pol>
struct ForceArgs {
    using pos_t = typename Pol::pos_t;
    using mass_t = typename Pol::mass_t;
    using calc_t = typename Pol::calc_t;
    const pos_t *xi, *yi, *zi;
    const pos_t *xj, *yj, *zj;
    const mass_t* mj;
    const mass_t* mi;     // masses of the sinks (self set only, for the potential)
    int ni, nj;
    int jspan;            // sources per j-split range, a multiple of BS
    calc_t eps2;
    double G;
    int self_pot;         // remove the j = i term m_i / eps from the potential
    pos_t *ax, *ay, *az, *pot;  // final outputs (part == nullptr)
    pos_t *vx, *vy, *vz;  // velocities to kick, or nullptr
    double h;             // kick: v <- v + h a, with a as stored
    pos_t *dx, *dy, *dz;  // with vx: positions of the next step's drift, or nullptr
    double dt;            // drift: v <- v + h a; x <- x + dt v (after the kick)
    double* part;         // [nsplit][NQ][ni] FP64 partial sums, or nullptr
};

template <class Pol, bool POT>
__device__ __forceinline__ void finish_sink(const ForceArgs<Pol>& a, int i, double sx, double sy,
                                            double sz, double sp) {
    using pos_t = typename Pol::pos_t;
    using calc_t = typename Pol::calc_t;
    const pos_t ax = pos_t(a.G * sx), ay = pos_t(a.G * sy), az = pos_t(a.G * sz);
    a.ax[i] = ax;
    a.ay[i] = ay;
    a.az[i] = az;
    if (a.vx) {  // the leapfrog's closing half-kick, same arithmetic as the kick kernel
        const pos_t h = pos_t(a.h);
        pos_t vx = fmat(h, ax, a.vx[i]), vy = fmat(h, ay, a.vy[i]), vz = fmat(h, az, a.vz[i]);
        if (a.dx) {  // and the next step's kick and drift, as the kick-drift kernel does them
            const pos_t dt = pos_t(a.dt);
            vx = fmat(h, ax, vx);
            vy = fmat(h, ay, vy);
            vz = fmat(h, az, vz);
            a.dx[i] = fmat(dt, vx, a.dx[i]);
            a.dy[i] = fmat(dt, vy, a.dy[i]);
            a.dz[i] = fmat(dt, vz, a.dz[i]);
        }
        a.vx[i] = vx;
        a.vy[i] = vy;
        a.vz[i] = vz;
    }
    if (POT) {
        double self = 0.0;
        if (a.self_pot) {
            // the j = i term exactly as the pair loop added it
            typename Pol::sum_t t;
            t.init();
            t.add_fma(calc_t(a.mi[i]), rsqrt_pair(a.eps2));
            self = t.total();
        }
        a.pot[i] = pos_t(-a.G * (sp - self));
    }
}

template <class Pol, int BS, int K, bool ACC, bool POT>
__global__ __launch_bounds__(BS) void force_kernel(ForceArgs<Pol> a) {
    using calc_t = typename Pol::calc_t;
    using sum_t = typename Pol::sum_t;
    using V4 = typename Vec4<calc_t>::type;
    __shared__ V4 tile[BS];

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
            if (i < a.ni) {
                cx += a.xi[i];
                cy += a.yi[i];
                cz += a.zi[i];
            }
        }
        sink_block_origin<BS / 64>(cx, cy, cz, min(a.ni - b0, BS * K), org, ox, oy, oz);
    }
    calc_t xi[K], yi[K], zi[K];
    sum_t sx[K], sy[K], sz[K], sp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k * BS;
        const bool ok = i < a.ni;
        xi[k] = ok ? pair_coord<Pol>(a.xi[i], ox) : calc_t(0);
        yi[k] = ok ? pair_coord<Pol>(a.yi[i], oy) : calc_t(0);
        zi[k] = ok ? pair_coord<Pol>(a.zi[i], oz) : calc_t(0);
        sx[k].init(); sy[k].init(); sz[k].init(); sp[k].init();
    }
    const calc_t eps2 = a.eps2;
    const int jbeg = blockIdx.y * a.jspan;
    const int jend = min(a.nj, jbeg + a.jspan);

    for (int jt = jbeg; jt < jend; jt += BS) {
        const int j = jt + tid;
        V4 p;
        if (j < jend) {
            p.x = pair_coord<Pol>(a.xj[j], ox);
            p.y = pair_coord<Pol>(a.yj[j], oy);
            p.z = pair_coord<Pol>(a.zj[j], oz);
            p.w = calc_t(a.mj[j]);
        } else {  // zero-mass padding: contributes exactly 0
            p.x = calc_t(0); p.y = calc_t(0); p.z = calc_t(0); p.w = calc_t(0);
        }
        __syncthreads();
        tile[tid] = p;
        __syncthreads();
#pragma unroll 8
        for (int jj = 0; jj < BS; ++jj) {
            const V4 q = tile[jj];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const calc_t dx = q.x - xi[k];
                const calc_t dy = q.y - yi[k];
                const calc_t dz = q.z - zi[k];
                const calc_t s = fmat(dz, dz, fmat(dy, dy, fmat(dx, dx, eps2)));
                const calc_t r = rsqrt_pair(s);
                if (ACC) {
                    calc_t w = r * (r * r);
                    w = w * q.w;
                    sx[k].add_fma(dx, w);
                    sy[k].add_fma(dy, w);
                    sz[k].add_fma(dz, w);
                }
                if (POT) sp[k].add_fma(q.w, r);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            sx[k].tile_end(); sy[k].tile_end(); sz[k].tile_end(); sp[k].tile_end();
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + k * BS;
        if (i >= a.ni) continue;
        if (a.part) {
            double* q = a.part + (size_t)blockIdx.y * NQ * a.ni;
            if (ACC) {
                q[i] = sx[k].total();
                q[(size_t)a.ni + i] = sy[k].total();
                q[(size_t)2 * a.ni + i] = sz[k].total();
            }
            if (POT) q[(size_t)3 * a.ni + i] = sp[k].total();
        } else if (ACC) {
            finish_sink<Pol, POT>(a, i, sx[k].total(), sy[k].total(), sz[k].total(), sp[k].total());
        }
    }
}

// Adds the nsplit partial sums of every sink in split order, then finishes.
template <class Pol, bool POT>
__global__ __launch_bounds__(256) void force_reduce_kernel(ForceArgs<Pol> a, int nsplit) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.ni) return;
    const size_t stride = (size_t)NQ * a.ni;
    double sx = 0, sy = 0, sz = 0, sp = 0;
    // eight ranges' loads in flight together, the adds in range order
#pragma unroll 8
    for (int s = 0; s < nsplit; ++s) {
        const double* q = a.part + s * stride;
        sx += q[i];
        sy += q[(size_t)a.ni + i];
        sz += q[(size_t)2 * a.ni + i];
        if (POT) sp += q[(size_t)3 * a.ni + i];
    }
    finish_sink<Pol, POT>(a, i, sx, sy, sz, sp);
}

template <class Pol>
ForceArgs<Pol> make_args(int64_t ni, const void* xi, int64_t nj, const void* xj, const void* mj,
                         double eps, double G, bool self_set, void* acc, void* pot) {
    using pos_t = typename Pol::pos_t;
    using mass_t = typename Pol::mass_t;
    using calc_t = typename Pol::calc_t;
    ForceArgs<Pol> a{};
    const pos_t* pi = static_cast<const pos_t*>(xi);
    const pos_t* pj = static_cast<const pos_t*>(xj);
    a.xi = pi; a.yi = pi + ni; a.zi = pi + 2 * ni;
    a.xj = pj; a.yj = pj + nj; a.zj = pj + 2 * nj;
    a.mj = static_cast<const mass_t*>(mj);
    a.mi = self_set ? a.mj : nullptr;
    a.ni = (int)ni;
    a.nj = (int)nj;
    a.eps2 = calc_t(eps) * calc_t(eps);
    a.G = G;
    a.self_pot = (self_set && pot) ? 1 : 0;
    pos_t* po = static_cast<pos_t*>(acc);
    if (po) { a.ax = po; a.ay = po + ni; a.az = po + 2 * ni; }
    a.pot = static_cast<pos_t*>(pot);
    return a;
}

int split_span(int64_t nj, int split, int block) {
    int64_t per = (nj + split - 1) / split;
    per = (per + block - 1) / block * block;
    return (int)per;
}

template <class Pol, bool ACC, bool POT, int BS, int K>
hipError_t launch_shape(ForceArgs<Pol> a, int nsplit, hipStream_t stream) {
    dim3 grid((a.ni + BS * K - 1) / (BS * K), nsplit);
    hipLaunchKernelGGL((force_kernel<Pol, BS, K, ACC, POT>), grid, dim3(BS), 0, stream, a);
    return hipGetLastError();
}

template <class Pol, bool ACC, bool POT>
hipError_t launch_any(const Shape& sh, ForceArgs<Pol> a, int nsplit, hipStream_t stream) {
#define NB_FORCE_CASE(BSV, KV) \
    if (sh.block == BSV && sh.ipl == KV) return launch_shape<Pol, ACC, POT, BSV, KV>(a, nsplit, stream);
    NB_FORCE_CASE(64, 1) NB_FORCE_CASE(64, 2) NB_FORCE_CASE(64, 4)
    NB_FORCE_CASE(128, 1) NB_FORCE_CASE(128, 2) NB_FORCE_CASE(128, 4)
    NB_FORCE_CASE(256, 1) NB_FORCE_CASE(256, 2) NB_FORCE_CASE(256, 4)
    NB_FORCE_CASE(512, 1) NB_FORCE_CASE(512, 2) NB_FORCE_CASE(512, 4)
    NB_FORCE_CASE(1024, 1) NB_FORCE_CASE(1024, 2) NB_FORCE_CASE(1024, 4)
#undef NB_FORCE_CASE
    return hipErrorInvalidValue;
}

template <class Pol, bool ACC, bool POT>
hipError_t run_force(const Shape& sh, ForceArgs<Pol> a, void* ws, bool partials_only,
                     hipStream_t stream, bool* drifted = nullptr) {
    const int span = split_span(a.nj, sh.split, sh.block);
    const int nsplit = (a.nj + span - 1) / span;
    a.jspan = span;
    if (nsplit == 1 && !partials_only) {
        // each workgroup finishes its own sinks while others may still read
        // their positions as sources: no drift here
        a.dx = a.dy = a.dz = nullptr;
        if (drifted) *drifted = false;
        a.part = nullptr;
        return launch_any<Pol, ACC, POT>(sh, a, 1, stream);
    }
    if (drifted) *drifted = a.dx != nullptr;
    a.part = static_cast<double*>(ws);
    hipError_t e = launch_any<Pol, ACC, POT>(sh, a, nsplit, stream);
    if (e != hipSuccess || partials_only) return e;
    hipLaunchKernelGGL((force_reduce_kernel<Pol, POT>), dim3((a.ni + 255) / 256), dim3(256), 0,
                       stream, a, nsplit);
    return hipGetLastError();
}

}  // namespace

bool shape_supported(const Shape& s) {
    const bool bs_ok = s.block == 64 || s.block == 128 || s.block == 256 || s.block == 512 ||
                       s.block == 1024;
    const bool k_ok = s.ipl == 1 || s.ipl == 2 || s.ipl == 4;
    return bs_ok && k_ok && s.split >= 1 && s.split <= 256;
}

size_t force_partials_bytes(const Shape& s, int64_t ni) {
    return (size_t)s.split * NQ * (size_t)ni * sizeof(double);
}

// Upper bound of force_partials_bytes(choose_force_shape(prec, ni, nj), ni)
// over every ni, nj <= n (a small sink set against a large source set takes
// the most ranges). From the rule below:
//  * a range is at least 4 tiles of >= 128 sources, or 8 of 64, i.e. >= 512
//    sources, except that below 16384 sources ranges as short as one tile
//    are allowed, at most 64 of them: split <= max(n/512, min(64, nj/64));
//  * split <= 256;
//  * split > 1 only while waves < 65536, where split <= 65536/waves + 1 and
//    ni <= waves * 64 * ipl, so split * ni < 2^23 * ipl <= 2^24 for the
//    shapes with ipl <= 2; the shape with ipl = 4 serves fewer than 65536
//    sinks, so there split * ni <= 256 * 65536 = 2^24 as well.
size_t force_partials_bound(int64_t n) {
    const int64_t short_ranges = std::min<int64_t>(64, std::min<int64_t>(n, 16383) / 64);
    const int64_t split = std::min<int64_t>(256, std::max<int64_t>(n / 512, short_ranges));
    if (split <= 1) return 0;
    const int64_t rows = std::min<int64_t>(split * n, int64_t(1) << 24);  // split * ni
    return (size_t)rows * NQ * sizeof(double);
}

Shape choose_force_shape(int prec, int64_t ni, int64_t nj) {
    // Measured on MI355X (launch-shape sweeps at N = 2^10 .. 2^20):
    //  * FP32 pair arithmetic: 1 sink per lane in 256-lane workgroups up to
    //    12288 sinks, then 2 sinks per lane, 128-lane workgroups, and
    //    512-lane ones (fewer barriers per pair) from 65536 sinks up;
    //  * FP64: 64-lane workgroups below 65536 sinks (1 sink per lane below
    //    3072, else 4), 256 lanes above;
    //  * many more workgroups than the chip holds at once balance the CUs
    //    better even when one round would already fill every SIMD: split the
    //    source range until there are ~64K wavefronts (8 ranges at 2^20, 32
    //    at 2^18, 5-16 % faster), keeping every range >= 4 tiles long (8
    //    for the 64-lane FP64 shape) -- or, below 16384 sources, as short as
    //    one tile, up to 32 ranges (64 in FP64): 6x faster at N = 1024 in
    //    FP64, 2.6x at 4096 in FP32, where the pass is otherwise a handful
    //    of workgroups.
    Shape s;
    if (prec == NB_F64) {
        s = ni < 3072 ? Shape{1, 64, 1} : (ni < 65536 ? Shape{4, 64, 1} : Shape{1, 256, 1});
    } else {
        s = ni <= 12288 ? Shape{1, 256, 1} : Shape{2, ni >= 65536 ? 512 : 128, 1};
    }
    const int64_t groups = (ni + (int64_t)s.block * s.ipl - 1) / ((int64_t)s.block * s.ipl);
    const int64_t waves = groups * (s.block / 64);
    const int64_t want = 65536;
    int64_t split = (want + waves - 1) / waves;
    const int64_t min_tiles = (prec == NB_F64 && s.block == 64) ? 8 : 4;
    const int64_t long_ranges = nj / (min_tiles * (int64_t)s.block);
    const int64_t short_ranges =
        nj < 16384 ? std::min<int64_t>(prec == NB_F64 ? 64 : 32, nj / (int64_t)s.block) : 0;
    const int64_t max_ranges = std::max(long_ranges, short_ranges);
    if (split > max_ranges) split = max_ranges;
    if (split > 256) split = 256;
    if (split < 1) split = 1;
    s.split = (int)split;
    return s;
}

hipError_t launch_force(int prec, const Shape& shape, int64_t ni, const void* xi, int64_t nj,
                        const void* xj, const void* mj, double eps, double G, bool self_set,
                        void* acc, void* pot, void* ws, hipStream_t stream, void* kick_v,
                        double kick_h, void* drift_x, double drift_dt, bool* drifted) {
    hipError_t err = hipErrorInvalidValue;
    if (drifted) *drifted = false;
    dispatch_prec(prec, [&](auto tag) {
        using Pol = decltype(tag);
        using pos_t = typename Pol::pos_t;
        auto a = make_args<Pol>(ni, xi, nj, xj, mj, eps, G, self_set, acc, pot);
        if (kick_v) {
            pos_t* pv = static_cast<pos_t*>(kick_v);
            a.vx = pv;
            a.vy = pv + ni;
            a.vz = pv + 2 * ni;
            a.h = kick_h;
            if (drift_x && self_set) {
                pos_t* px = static_cast<pos_t*>(drift_x);
                a.dx = px;
                a.dy = px + ni;
                a.dz = px + 2 * ni;
                a.dt = drift_dt;
            }
        }
        err = pot ? run_force<Pol, true, true>(shape, a, ws, false, stream, drifted)
                  : run_force<Pol, true, false>(shape, a, ws, false, stream, drifted);
    });
    return err;
}

}  // namespace nb
