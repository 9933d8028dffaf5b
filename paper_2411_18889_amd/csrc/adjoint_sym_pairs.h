// The pair kernel of the symmetric adjoint pass (the description is in
// adjoint_sym.hip), shared by the two translation units that instantiate it:
// adjoint_sym.hip the passes that also sum the force, adjoint_sym_entry.hip
// the force-free passes, which are built with another instruction schedule.
#pragma once

#include "common.h"

namespace nb {
namespace asym {

constexpr int TJ = 128;  // sources per LDS tile
constexpr int NQ = 7;

// One band of the pair pass, as the symmetric force pass (SymLayout): the
// items of rows I0 <= I < I1; NQF partial rows per particle and slot, in the
// policy's pair type (FP32; FP64 for the FP64 policy).
template <class Pol>
struct ASymArgs {
    using pos_t = typename Pol::pos_t;
    using mass_t = typename Pol::mass_t;
    using calc_t = typename Pol::calc_t;
    const pos_t *x, *y, *z;
    const mass_t* m;
    const pos_t *lx, *ly, *lz;  // lam_v
    int n, nb;
    SymBandView band;
    calc_t eps2;
    calc_t* part;  // the band's partials (SymBandView::offset)
};

// F: also accumulate the force a (quantities 0..2); without it (a pass whose
// state comes from a checkpoint, not from walking back) the quantities are
// 3..6 only: 8 VALU, three rotations and three partial rows less per pair.
template <bool F> struct QRange {
    static constexpr int lo = F ? 0 : 3;  // first quantity accumulated
    static constexpr int n = NQ - lo;     // partial rows per block
};

template <int K, bool JSIDE, bool F, class Sum, class C, class V4>
__device__ __forceinline__ void asym_tile(const V4 (*rp)[128], const V4 (*rl)[128], C* jq,
                                          const C* xi, const C* yi, const C* zi, const C* mi,
                                          const C* mi3, const C* lxi, const C* lyi, const C* lzi,
                                          Sum (*s)[NQ], C eps2, int lane) {
    // groups of 64 sources stored twice in a row: lane l reads source
    // (l + t) mod 64 at rp[g][l + t] (see the force pass)
    for (int g = 0; g < TJ / 64; ++g) {
        const V4* rowp = rp[g] + lane;
        const V4* rowl = rl[g] + lane;
        // j-side sums of the group's sources, carried one lane down per step
        constexpr int Q0 = QRange<F>::lo;
        C c[NQ];
#pragma unroll
        for (int p = Q0; p < NQ; ++p) c[p] = C(0);
        // two steps per iteration for the force-free passes (their schedule
        // interleaves the sinks, adjoint_sym_entry.hip), one for the passes
        // with the force sums, which then run about 4 % faster (2^20: 477
        // against 497 ms; 262144: 30.0 against 31.3; 16384: 0.192 against
        // 0.205; the force-free passes unchanged; one box)
#pragma unroll(F ? 1 : 2)
        for (int t = 0; t < 64; ++t) {
            const V4 q = rowp[t];
            const V4 lj = rowl[t];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const C dx = q.x - xi[k];
                const C dy = q.y - yi[k];
                const C dz = q.z - zi[k];
                const C ss = fmat(dz, dz, fmat(dy, dy, fmat(dx, dx, eps2)));
                const C r = rsqrt_pair(ss);
                const C r2 = r * r;
                const C r3 = r2 * r;
                if (F) {
                    const C wj = r3 * q.w;
                    s[k][0].add_fma(dx, wj);
                    s[k][1].add_fma(dy, wj);
                    s[k][2].add_fma(dz, wj);
                }
                const C ux = fmat(mi[k], lj.x, -(q.w * lxi[k]));
                const C uy = fmat(mi[k], lj.y, -(q.w * lyi[k]));
                const C uz = fmat(mi[k], lj.z, -(q.w * lzi[k]));
                const C dl = fmat(dz, lj.z, fmat(dy, lj.y, dx * lj.x));  // d . lam_j
                C e, dli = C(0);
                if (JSIDE) {
                    // -3 d . u = (-3 m_i)(d . lam_j) - (-3 m_j)(d . lam_i): both dots are
                    // needed anyway, and the factors -3 m come with the sink and the
                    // source record
                    dli = fmat(dz, lzi[k], fmat(dy, lyi[k], dx * lxi[k]));
                    e = r2 * fmat(mi3[k], dl, -(lj.w * dli));
                } else {
                    e = (C(-3) * r2) * fmat(dz, uz, fmat(dy, uy, dx * ux));
                }
                const C tx = fmat(e, dx, ux);
                const C ty = fmat(e, dy, uy);
                const C tz = fmat(e, dz, uz);
                s[k][3].add_fma(r3, tx);
                s[k][4].add_fma(r3, ty);
                s[k][5].add_fma(r3, tz);
                s[k][6].add_fma(r3, dl);
                if (JSIDE) {
                    if (F) {
                        const C wi = r3 * mi[k];
                        c[0] = fmat(dx, wi, c[0]);
                        c[1] = fmat(dy, wi, c[1]);
                        c[2] = fmat(dz, wi, c[2]);
                    }
                    c[3] = fmat(r3, tx, c[3]);
                    c[4] = fmat(r3, ty, c[4]);
                    c[5] = fmat(r3, tz, c[5]);
                    c[6] = fmat(r3, dli, c[6]);
                }
            }
            if (JSIDE) {
#pragma unroll
                for (int p = Q0; p < NQ; ++p) c[p] = from_next_lane(c[p]);
            }
        }
        if (JSIDE) {  // back in the lane that owns the source
#pragma unroll
            for (int p = Q0; p < NQ; ++p) jq[p * TJ + g * 64 + lane] = c[p];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int p = Q0; p < NQ; ++p) s[k][p].tile_end();
    }
}

template <class Pol, int W, int K, bool F>
__global__ __launch_bounds__(W * 64) void adjoint_sym_kernel(ASymArgs<Pol> a) {
    using C = typename Pol::calc_t;
    using V4 = typename Vec4<C>::type;
    constexpr int Q0 = QRange<F>::lo, NQF = QRange<F>::n;
    constexpr int NT = W * 64;
    constexpr int BI = NT * K;
    static_assert(BI % TJ == 0, "a block must hold whole tiles");
    __shared__ V4 rp[TJ / 64][128];
    __shared__ V4 rl[TJ / 64][128];
    __shared__ C jacc[W][NQ][TJ];

    int I, J;
    band_item(blockIdx.x, a.band.I0, a.band.I1, I, J);
    const bool jside = I != J;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int ibase = I * BI + w * 64 * K + lane;
    // origin of the pair arithmetic (tile-compensated policy): the centroid
    // of block I (see sink_block_origin), for both ends of every pair of the
    // item
    double ox = 0.0, oy = 0.0, oz = 0.0;
    if constexpr (Pol::origin) {
        __shared__ double org[W][3];
        double cx = 0.0, cy = 0.0, cz = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = ibase + k * 64;
            if (i < a.n) {
                cx += a.x[i];
                cy += a.y[i];
                cz += a.z[i];
            }
        }
        sink_block_origin<W>(cx, cy, cz, min(a.n - I * BI, BI), org, ox, oy, oz);
    }
    C xi[K], yi[K], zi[K], mi[K], mi3[K], lxi[K], lyi[K], lzi[K];
    // the sink side: the policy's sum; tile-compensated with four sinks per
    // lane (registers are short) an FP32 running sum over the block, as the
    // source side is
    using Sum = typename std::conditional<(K > 2 && std::is_same<typename Pol::sum_t, SumTile>::value),
                                          SumPlain<float>, typename Pol::sum_t>::type;
    Sum s[K][NQ];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ibase + k * 64;
        const bool ok = i < a.n;
        xi[k] = ok ? pair_coord<Pol>(a.x[i], ox) : C(0);
        yi[k] = ok ? pair_coord<Pol>(a.y[i], oy) : C(0);
        zi[k] = ok ? pair_coord<Pol>(a.z[i], oz) : C(0);
        mi[k] = ok ? C(a.m[i]) : C(0);  // a padding sink adds exactly 0 to the j side
        mi3[k] = C(-3) * mi[k];
        lxi[k] = ok ? C(a.lx[i]) : C(0);
        lyi[k] = ok ? C(a.ly[i]) : C(0);
        lzi[k] = ok ? C(a.lz[i]) : C(0);
#pragma unroll
        for (int p = Q0; p < NQ; ++p) s[k][p].init();
    }

    const int jb = J * BI;
    const int je = min(a.n, jb + BI);
    for (int jt = jb; jt < je; jt += TJ) {
        for (int q = tid; q < TJ; q += NT) {
            const int j = jt + q;
            V4 p, l;  // zero mass and adjoint past the end: adds 0
            p.x = p.y = p.z = p.w = l.x = l.y = l.z = l.w = C(0);
            if (j < je) {
                p.x = pair_coord<Pol>(a.x[j], ox);
                p.y = pair_coord<Pol>(a.y[j], oy);
                p.z = pair_coord<Pol>(a.z[j], oz);
                p.w = C(a.m[j]);
                l.x = C(a.lx[j]);
                l.y = C(a.ly[j]);
                l.z = C(a.lz[j]);
                l.w = C(-3) * C(a.m[j]);
            }
            rp[q >> 6][q & 63] = p;
            rp[q >> 6][(q & 63) + 64] = p;
            rl[q >> 6][q & 63] = l;
            rl[q >> 6][(q & 63) + 64] = l;
        }
        __syncthreads();
        if (jside)
            asym_tile<K, true, F, Sum, C, V4>(rp, rl, &jacc[w][0][0], xi, yi, zi, mi, mi3, lxi,
                                              lyi, lzi, s, a.eps2, lane);
        else
            asym_tile<K, false, F, Sum, C, V4>(rp, rl, nullptr, xi, yi, zi, mi, mi3, lxi, lyi,
                                               lzi, s, a.eps2, lane);
        __syncthreads();
        if (jside) {
            for (int q = tid; q < NQF * TJ; q += NT) {
                const int r = q / TJ, jj = q - r * TJ;  // partial row r = quantity Q0 + r
                C sum = C(0);
#pragma unroll
                for (int v = 0; v < W; ++v) sum += jacc[v][Q0 + r][jj];
                const int j = jt + jj;
                // slot I of particle j
                if (j < je) a.part[a.band.offset(I, r, j)] = -sum;
            }
        }
    }
    // slot J of the sinks of block I
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ibase + k * 64;
        if (i >= a.n) continue;
#pragma unroll
        for (int p = Q0; p < NQ; ++p) a.part[a.band.offset(J, p - Q0, i)] = C(s[k][p].total());
    }
}

// One band of the pair pass in shape W x K; F: with the force sums.
template <class Pol, int W, int K, bool F>
hipError_t launch_pairs(const ASymArgs<Pol>& a, hipStream_t stream) {
    const int64_t R = a.band.I1 - a.band.I0;
    const int64_t items = R * (R + 1) / 2 + R * (a.nb - a.band.I1);  // < 2^31 / threads (sym_band_end)
    hipLaunchKernelGGL((adjoint_sym_kernel<Pol, W, K, F>), dim3((unsigned)items), dim3(W * 64), 0,
                       stream, a);
    return hipGetLastError();
}

// The force-free pair pass of one band (adjoint_sym_entry.hip).
hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs<PolMixTileC>& a,
                              hipStream_t stream);
hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs<PolF32>& a, hipStream_t stream);
hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs<PolF64>& a, hipStream_t stream);

}  // namespace asym
}  // namespace nb
