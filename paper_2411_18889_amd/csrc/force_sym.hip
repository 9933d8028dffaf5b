// Symmetric pair-force pass of Eq. (1) for one particle set acting on itself
// (the tile-compensated, plain FP32 and FP64 policies), on gfx950.
//
// Newton's third law: the pair (i, j) exerts m_j d s^-3/2 on i and
// -m_i d s^-3/2 on j (d = x_j - x_i), so one reciprocal square root and one
// s^-3/2 serve both bodies: 16 VALU + 1 rsqrt per pair, i.e. 8 VALU + 1/2
// rsqrt per interaction against 12 + 1 for the one-sided kernel. The cost is
// that the j side has to be summed across lanes and workgroups; it is done
// here in a fixed order, without global atomics, so the result is bitwise
// reproducible:
//
//  * the particles are cut into nb blocks of BI = W*64*K; a work item is a
//    block pair (I, J) with I <= J (nb (nb + 1) / 2 items, one workgroup each);
//  * item (I, J), I < J: lane l of wave w holds K sinks of block I in
//    registers; the sources of block J are staged in LDS tiles of TJ, and in
//    every 64-source group lane l meets source (l + t) mod 64 at step t, so
//    the 64 lanes touch 64 different sources at every step. The i side is a
//    running FP32 sum folded into FP64 after each group (as the tile-
//    compensated policy) where a lane holds up to four sinks, and an FP32
//    sum over the whole source block, as the j side's, where it holds eight
//    (registers are short); the j-side sum of a source travels with it through
//    the lanes (a one-lane rotation per step through the LDS crossbar), so
//    after the 64 steps of a group it is back in the lane that owns the
//    source, which writes it to the wave's LDS row. At the end of a tile the
//    W wave rows are added in wave order;
//  * item (I, I): the block on itself, i side only (each pair from both
//    ends, the j = i term contributing 0);
//  * every item writes FP32 partials: its i side for block I into slot J, its
//    j side for block J into slot I. Each particle of block P so receives
//    exactly one partial in each slot k = 0 .. nb-1 (k < P: j side of item
//    (k, P); k = P: item (P, P); k > P: i side of item (P, k)), and a second
//    kernel adds the nb slots in slot order in FP64, then applies G and the
//    optional closing half-kick. The items run in bands of rows I, each band
//    followed by a kernel that folds the slots it wrote into running sums
//    (SymLayout): the sums are bitwise those of one launch, and the scratch
//    is one band's partials;
//  * with the potential, the same reciprocal square root also gives the
//    fourth quantity: m_j / r on the i side and m_i / r on the j side (no
//    sign change, the potential is symmetric). The diagonal items include
//    the j = i term m_i / eps, which the finish kernel removes with the same
//    product the pair loop formed.
//  * three policies use it: the tile-compensated one (FP64 state, FP32 pair
//    arithmetic on positions taken relative to the centroid of block I, see
//    sink_block_origin; each group's FP32 i-side sum folded into FP64; FP32
//    partials added in FP64), plain FP32 (FP32 state; the i-side a running
//    FP32 sum over the whole source block; the slots added in FP32: every
//    sum stays FP32, as the policy asks, only blocked by the third-law
//    structure) and FP64 (FP64 records, pair arithmetic, source-side sums,
//    partials and slot sums; the source-side sums rotate as two 32-bit
//    halves). The description above says FP32 where it is the pair type.
//
// The build compiles this file with LLVM's iterative ILP scheduling strategy
// (-mllvm -amdgpu-sched-strategy=iterative-ilp), measured against the default
// on one box: tile-compensated 2^20 186.0 against 188.9 ms (with the
// potential 206.7 against 207.9), plain FP32 186.4 against 188.8, 262144 12.10
// against 12.23 ms, FP64 and 65536 unchanged.
#include "common.h"

namespace nb {

namespace {

constexpr int TJ = 256;  // sources per LDS tile

// pos_t / mass_t: state and mass types; calc_t: pair arithmetic (also the
// source-side sums and the partials); sum_t: per-sink i-side sum; fin_t:
// type the finishing kernel adds the slots in.
template <class Pos, class Mass, class Calc, class Sum, class Fin>
struct SymPol {
    using pos_t = Pos;
    using mass_t = Mass;
    using calc_t = Calc;
    using sum_t = Sum;
    using fin_t = Fin;
    // FP64 state, FP32 pairs: positions relative to the sink block's centroid
    static constexpr bool origin =
        std::is_same<Pos, double>::value && std::is_same<Calc, float>::value;
};
using SymTileC = SymPol<double, float, float, SumTile, double>;
using SymF32 = SymPol<float, float, float, SumPlain<float>, float>;
using SymF64 = SymPol<double, double, double, SumPlain<double>, double>;

// One band of the pair pass: the items of rows I0 <= I < I1 (see SymLayout).
// NQ = 3 partial quantities, or 4 with the potential.
template <class Pol>
struct SymArgs {
    const typename Pol::pos_t *x, *y, *z;
    const typename Pol::mass_t* m;
    int n, nb;
    SymBandView band;
    typename Pol::calc_t eps2;
    typename Pol::calc_t* part;  // the band's partials (SymBandView::offset)
};

// The fold of one band: particles base .. n-1 add their slots I0 .. I1-1;
// the band's own particles also their slots I1 .. nb-1, and are finished;
// the others keep their running sums for the next band.
template <class Pol>
struct SymFinishArgs {
    const typename Pol::calc_t* part;  // the band's partials
    SymBandView band;
    typename Pol::fin_t* run;       // [NQ][n] running sums between bands, or nullptr
    int first;                      // the first band: the sums start at 0
    const typename Pol::mass_t* m;  // for the j = i potential term
    int n, nb;
    typename Pol::calc_t eps2;
    double G;
    typename Pol::pos_t *ax, *ay, *az;
    typename Pol::pos_t* pot;           // or nullptr
    typename Pol::pos_t *vx, *vy, *vz;  // or nullptr
    double h;
    typename Pol::pos_t *dx, *dy, *dz;  // with vx: the next step's drift, or nullptr
    double dt;
};

// One tile of sources against the K sinks of this lane. The tile is held as
// TJ/64 groups of 64 sources, each stored twice in a row (rec[g][0..127]), so
// that lane l meets source (l + t) mod 64 of the group at step t by reading
// rec[g][l + t]: the step is an immediate offset of the LDS read. The j-side
// sums of the group travel with their source, one lane down per step, so
// after 64 steps lane l holds the sum of source l, which it stores in the
// wave's LDS row jq[c][g*64 + l]. P adds the potential as a fourth quantity.
template <int K, bool JSIDE, bool P, class Sum, class C>
__device__ __forceinline__ void sym_tile(const typename Vec4<C>::type (*rec)[128], C* jq,
                                         const C* xi, const C* yi, const C* zi, const C* mi,
                                         Sum (*s)[4], C eps2, int lane) {
    for (int g = 0; g < TJ / 64; ++g) {
        const typename Vec4<C>::type* row = rec[g] + lane;
        C cx = C(0), cy = C(0), cz = C(0), cp = C(0);
#pragma unroll 4
        for (int t = 0; t < 64; ++t) {
            const typename Vec4<C>::type q = row[t];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const C dx = q.x - xi[k];
                const C dy = q.y - yi[k];
                const C dz = q.z - zi[k];
                const C ss = fmat(dz, dz, fmat(dy, dy, fmat(dx, dx, eps2)));
                const C r = rsqrt_pair(ss);
                const C r3 = r * (r * r);
                const C wj = r3 * q.w;
                s[k][0].add_fma(dx, wj);
                s[k][1].add_fma(dy, wj);
                s[k][2].add_fma(dz, wj);
                if (P) s[k][3].add_fma(q.w, r);
                if (JSIDE) {
                    const C wi = r3 * mi[k];
                    cx = fmat(dx, wi, cx);
                    cy = fmat(dy, wi, cy);
                    cz = fmat(dz, wi, cz);
                    if (P) cp = fmat(mi[k], r, cp);
                }
            }
            if (JSIDE) {
                cx = from_next_lane(cx);
                cy = from_next_lane(cy);
                cz = from_next_lane(cz);
                if (P) cp = from_next_lane(cp);
            }
        }
        if (JSIDE) {
            jq[g * 64 + lane] = cx;
            jq[TJ + g * 64 + lane] = cy;
            jq[2 * TJ + g * 64 + lane] = cz;
            if (P) jq[3 * TJ + g * 64 + lane] = cp;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            s[k][0].tile_end();
            s[k][1].tile_end();
            s[k][2].tile_end();
            if (P) s[k][3].tile_end();
        }
    }
}

template <class Pol, int W, int K, bool P>
__global__ __launch_bounds__(W * 64) void force_sym_kernel(SymArgs<Pol> a) {
    using C = typename Pol::calc_t;
    using V4 = typename Vec4<C>::type;
    constexpr int NT = W * 64;
    constexpr int BI = NT * K;
    constexpr int NQ = P ? 4 : 3;
    static_assert(BI % TJ == 0, "a block must hold whole tiles");
    __shared__ V4 rec[TJ / 64][128];
    __shared__ C jacc[W][NQ][TJ];

    int I, J;
    band_item(blockIdx.x, a.band.I0, a.band.I1, I, J);
    const bool jside = I != J;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int ibase = I * BI + w * 64 * K + lane;
    // origin of the pair arithmetic (tile-compensated policy): the centroid
    // of block I, for both ends of every pair of the item
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
    C xi[K], yi[K], zi[K], mi[K];
    // the sink side: the policy's sum; with eight sinks per lane (registers
    // are short) an FP32 running sum over the block, as the source side is
    using Sum = typename std::conditional<(K > 4 && std::is_same<typename Pol::sum_t, SumTile>::value),
                                          SumPlain<float>, typename Pol::sum_t>::type;
    Sum s[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ibase + k * 64;
        const bool ok = i < a.n;
        xi[k] = ok ? pair_coord<Pol>(a.x[i], ox) : C(0);
        yi[k] = ok ? pair_coord<Pol>(a.y[i], oy) : C(0);
        zi[k] = ok ? pair_coord<Pol>(a.z[i], oz) : C(0);
        mi[k] = ok ? C(a.m[i]) : C(0);  // a padding sink adds exactly 0 to the j side
        s[k][0].init();
        s[k][1].init();
        s[k][2].init();
        s[k][3].init();
    }

    const int jb = J * BI;
    const int je = min(a.n, jb + BI);
    for (int jt = jb; jt < je; jt += TJ) {
        for (int q = tid; q < TJ; q += NT) {
            const int j = jt + q;
            V4 p;  // zero-mass padding past the end
            p.x = j < je ? pair_coord<Pol>(a.x[j], ox) : C(0);
            p.y = j < je ? pair_coord<Pol>(a.y[j], oy) : C(0);
            p.z = j < je ? pair_coord<Pol>(a.z[j], oz) : C(0);
            p.w = j < je ? C(a.m[j]) : C(0);
            rec[q >> 6][q & 63] = p;
            rec[q >> 6][(q & 63) + 64] = p;
        }
        __syncthreads();
        if (jside)
            sym_tile<K, true, P, Sum, C>(rec, &jacc[w][0][0], xi, yi, zi, mi, s,
                                                         a.eps2, lane);
        else
            sym_tile<K, false, P, Sum, C>(rec, nullptr, xi, yi, zi, mi, s,
                                                          a.eps2, lane);
        __syncthreads();
        if (jside) {
            // j side of this tile: the wave rows added in wave order (every
            // row entry is rewritten by the next tile before it is read again)
            // (the force on j is minus the sum, its potential the sum)
            for (int q = tid; q < NQ * TJ; q += NT) {
                const int c = q / TJ, jj = q - c * TJ;
                C sum = C(0);
#pragma unroll
                for (int v = 0; v < W; ++v) sum += jacc[v][c][jj];
                const int j = jt + jj;
                // slot I of particle j
                if (j < je) a.part[a.band.offset(I, c, j)] = c < 3 ? -sum : sum;
            }
        }
        // rec is rewritten only after every wave has passed the barrier above
    }
    // slot J of the sinks of block I
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = ibase + k * 64;
        if (i >= a.n) continue;
#pragma unroll
        for (int c = 0; c < NQ; ++c) a.part[a.band.offset(J, c, i)] = C(s[k][c].total());
    }
}

// The fold of one band (SymFinishArgs): adds a particle's partials in slot
// order (in fin_t: FP64 for the tile-compensated and FP64 policies, FP32 for
// the FP32 one) to its running sum; when its slots are complete, stores
// a = G * sum and applies the optional half-kick v <- v + h a, with a as
// stored; with P, also the potential -G (sum - m_i / eps).
template <class Pol, bool P>
__global__ __launch_bounds__(256) void force_sym_finish_kernel(SymFinishArgs<Pol> a) {
    using pos_t = typename Pol::pos_t;
    using fin_t = typename Pol::fin_t;
    using calc_t = typename Pol::calc_t;
    constexpr int NQ = P ? 4 : 3;
    const SymBandView& b = a.band;
    const int i = b.base + blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    fin_t sx = 0, sy = 0, sz = 0, sp = 0;
    if (!a.first) {
        sx = a.run[i];
        sy = a.run[(size_t)a.n + i];
        sz = a.run[(size_t)2 * a.n + i];
        if (P) sp = a.run[(size_t)3 * a.n + i];
    }
    // slots I0 .. I1-1 (region A), unrolled so that the loads of eight slots
    // are in flight together (the adds stay in slot order; at small n the
    // pass is latency-bound here)
#pragma unroll 8
    for (int k = b.I0; k < b.I1; ++k) {
        sx += fin_t(a.part[b.offset(k, 0, i)]);
        sy += fin_t(a.part[b.offset(k, 1, i)]);
        sz += fin_t(a.part[b.offset(k, 2, i)]);
        if (P) sp += fin_t(a.part[b.offset(k, 3, i)]);
    }
    if (i >= b.base + b.nbp) {  // a later band adds this particle's next slots
        a.run[i] = sx;
        a.run[(size_t)a.n + i] = sy;
        a.run[(size_t)2 * a.n + i] = sz;
        if (P) a.run[(size_t)3 * a.n + i] = sp;
        return;
    }
    // the band's own particles: slots I1 .. nb-1 (region B), then finish
#pragma unroll 8
    for (int k = b.I1; k < a.nb; ++k) {
        sx += fin_t(a.part[b.offset(k, 0, i)]);
        sy += fin_t(a.part[b.offset(k, 1, i)]);
        sz += fin_t(a.part[b.offset(k, 2, i)]);
        if (P) sp += fin_t(a.part[b.offset(k, 3, i)]);
    }
    if (P) {
        // the j = i term as the pair loop formed it: m_i times the
        // reciprocal square root of eps^2, one product in the pair type
        const double self = double(a.m[i] * rsqrt_pair(a.eps2));
        a.pot[i] = pos_t(-a.G * (double(sp) - self));
    }
    const pos_t ax = pos_t(a.G * double(sx)), ay = pos_t(a.G * double(sy)),
                az = pos_t(a.G * double(sz));
    a.ax[i] = ax;
    a.ay[i] = ay;
    a.az[i] = az;
    if (a.vx) {  // the leapfrog's closing half-kick, in the state type
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
}

template <class Pol, int W, int K>
hipError_t launch_sym(const SymArgs<Pol>& a, bool pot, hipStream_t stream) {
    const int64_t R = a.band.I1 - a.band.I0;
    const int64_t items = R * (R + 1) / 2 + R * (a.nb - a.band.I1);  // < 2^31 / threads (sym_band_end)
    if (pot)
        hipLaunchKernelGGL((force_sym_kernel<Pol, W, K, true>), dim3((unsigned)items), dim3(W * 64),
                           0, stream, a);
    else
        hipLaunchKernelGGL((force_sym_kernel<Pol, W, K, false>), dim3((unsigned)items),
                           dim3(W * 64), 0, stream, a);
    return hipGetLastError();
}

template <class Pol>
hipError_t run_sym(const SymShape& sh, int64_t n, const void* x, const void* m, double eps,
                   double G, void* acc, void* ws, size_t ws_bytes, hipStream_t stream,
                   void* kick_v, double kick_h, void* pot, void* drift_x, double drift_dt) {
    using pos_t = typename Pol::pos_t;
    using calc_t = typename Pol::calc_t;
    using fin_t = typename Pol::fin_t;
    const int64_t bi = (int64_t)sh.waves * 64 * sh.ipl;
    const SymLayout L{n, bi, (int)((n + bi - 1) / bi), pot ? 4 : 3, sizeof(calc_t), sizeof(fin_t)};
    // one band when the workspace holds every partial; else the running sums
    // first, then one band's partials at a time
    const SymPlan plan = sym_plan(L, ws_bytes, sh.waves * 64);
    if (!plan.valid) return hipErrorInvalidValue;
    fin_t* run = plan.one ? nullptr : static_cast<fin_t*>(ws);
    calc_t* parts = reinterpret_cast<calc_t*>(static_cast<char*>(ws) + plan.parts);
    const size_t budget = plan.budget;

    SymArgs<Pol> a{};
    const pos_t* p = static_cast<const pos_t*>(x);
    a.x = p;
    a.y = p + n;
    a.z = p + 2 * n;
    a.m = static_cast<const typename Pol::mass_t*>(m);
    a.n = (int)n;
    a.nb = L.nb;
    a.eps2 = calc_t(eps) * calc_t(eps);
    SymFinishArgs<Pol> f{};
    f.run = run;
    f.m = a.m;
    f.n = a.n;
    f.eps2 = a.eps2;
    f.G = G;
    f.pot = static_cast<pos_t*>(pot);
    pos_t* po = static_cast<pos_t*>(acc);
    f.ax = po;
    f.ay = po + n;
    f.az = po + 2 * n;
    if (kick_v) {
        pos_t* pv = static_cast<pos_t*>(kick_v);
        f.vx = pv;
        f.vy = pv + n;
        f.vz = pv + 2 * n;
        f.h = kick_h;
        if (drift_x) {
            pos_t* px = static_cast<pos_t*>(drift_x);
            f.dx = px;
            f.dy = px + n;
            f.dz = px + 2 * n;
            f.dt = drift_dt;
        }
    }
    a.part = parts;
    f.part = parts;
    f.nb = L.nb;
    for (int I0 = 0; I0 < L.nb;) {
        const int I1 = sym_band_end(L, I0, budget, sh.waves * 64);
        a.band = f.band = sym_band_view(L, I0, I1);
        hipError_t e = hipErrorInvalidValue;
#define NB_SYM_CASE(WV, KV) \
    if (sh.waves == WV && sh.ipl == KV) e = launch_sym<Pol, WV, KV>(a, pot != nullptr, stream);
        NB_SYM_CASE(2, 2) NB_SYM_CASE(4, 2) NB_SYM_CASE(8, 2) NB_SYM_CASE(16, 2)
        NB_SYM_CASE(2, 4) NB_SYM_CASE(4, 4) NB_SYM_CASE(8, 4) NB_SYM_CASE(16, 4)
        NB_SYM_CASE(2, 8) NB_SYM_CASE(4, 8) NB_SYM_CASE(8, 8)
#undef NB_SYM_CASE
        if (e != hipSuccess) return e;
        f.first = I0 == 0;
        const dim3 fg((unsigned)((a.band.np + 255) / 256));
        if (pot)
            hipLaunchKernelGGL((force_sym_finish_kernel<Pol, true>), fg, dim3(256), 0, stream, f);
        else
            hipLaunchKernelGGL((force_sym_finish_kernel<Pol, false>), fg, dim3(256), 0, stream, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        I0 = I1;
    }
    return hipSuccess;
}

}  // namespace

bool sym_shape_supported(int prec, const SymShape& s) {
    if (prec != NB_MIX_TILEC && prec != NB_F32 && prec != NB_F64) return false;
    return ((s.ipl == 2 || s.ipl == 4) &&
            (s.waves == 2 || s.waves == 4 || s.waves == 8 || s.waves == 16)) ||
           (s.ipl == 8 && (s.waves == 2 || s.waves == 4 || s.waves == 8));
}

SymLayout sym_layout(int prec, const SymShape& s, int64_t n, bool pot) {
    const int64_t bi = (int64_t)s.waves * 64 * s.ipl;
    const size_t elem = prec == NB_F64 ? sizeof(double) : sizeof(float);  // partial type
    const size_t fin = prec == NB_F32 ? sizeof(float) : sizeof(double);   // running sum type
    return SymLayout{n, bi, (int)((n + bi - 1) / bi), pot ? 4 : 3, elem, fin};
}

SymShape choose_sym_shape(int prec, int64_t n, bool pot) {
    // Measured on MI355X with the tuner (tune.py; the run these figures come
    // from is in profiles/launch_shape_tuning.md), from 16384 to 2^21:
    //  * below 81920 particles two sinks per lane in blocks of at most n/48
    //    (>= 1176 equal work items for the 256 CUs): 256, or 512 from 24576
    //    (65536: 0.954 ms, the fastest shape 0.948);
    //  * from 81920 four-wave workgroups with four sinks per lane, blocks of
    //    1024 (81920: 1.292 against 1.347 ms for 4 x 2; 114688: 2.426 against
    //    2.580; 131072: 3.47 ms, the fastest symmetric shape);
    //  * from 2^18 four waves with eight sinks per lane, blocks of 2048: one
    //    LDS record read and three source-side rotations per eight pairs, and
    //    with FP32 block sums on the sink side 120 VGPRs (4 waves per SIMD)
    //    against 167 (3) for four sinks per lane -- 2^20: 204.5 ms against
    //    211.7 for 4 x 4, 2^18: 13.16 against 13.56; FP64 (FP64 sums
    //    throughout) 2^20: 436.2 ms against 477.5 for 8 waves x 4, 2^18: 27.6
    //    against 28.0 for 4 x 4.
    // Blocks of 2048 at every n from 2^18: eight waves in blocks of 4096
    // halve the partials but gain nothing (2^21: 814.2 ms against 815.5),
    // and with the potential (137 VGPRs, three waves per SIMD) a CU holds
    // only one eight-wave workgroup (2^21 with the potential: 1024 ms in
    // blocks of 4096, 835 in blocks of 2048). The partials (nb * 3 * n
    // values, nb * 4 * n with the potential) are written and folded in bands
    // of the workspace (SymLayout), so the pass serves every n up to 2^28 in
    // bounded memory.
    // Below 12288 particles the one-sided kernel is faster (measured, with the
    // finishing kernel's loads overlapped: one-sided 19 % faster at 8192;
    // symmetric 23 % faster at 12288, 37 % at 24576).
    if ((prec != NB_MIX_TILEC && prec != NB_F32 && prec != NB_F64) || n < 48 * 256 ||
        n > (int64_t(1) << 28))
        return SymShape{0, 0};
    auto bi = [](const SymShape& c) { return (int64_t)c.waves * 64 * c.ipl; };
    if (n < 81920) {
        static const SymShape small[] = {{2, 2}, {4, 2}};  // 256, 512
        return bi(small[1]) <= n / 48 ? small[1] : small[0];
    }
    (void)pot;  // the potential takes the same shapes
    if (n < (int64_t(1) << 18)) return SymShape{4, 4};  // 1024
    return SymShape{4, 8};                               // 2048
}

hipError_t launch_force_sym(int prec, const SymShape& sh, int64_t n, const void* x,
                            const void* m, double eps, double G, void* acc, void* ws,
                            size_t ws_bytes, hipStream_t stream, void* kick_v, double kick_h,
                            void* pot, void* drift_x, double drift_dt, bool* drifted) {
    if ((int64_t)sh.waves * sh.ipl == 0) return hipErrorInvalidValue;
    if (!kick_v) drift_x = nullptr;
    if (drifted) *drifted = drift_x != nullptr;
    if (prec == NB_MIX_TILEC)
        return run_sym<SymTileC>(sh, n, x, m, eps, G, acc, ws, ws_bytes, stream, kick_v, kick_h,
                                 pot, drift_x, drift_dt);
    if (prec == NB_F32)
        return run_sym<SymF32>(sh, n, x, m, eps, G, acc, ws, ws_bytes, stream, kick_v, kick_h,
                               pot, drift_x, drift_dt);
    if (prec == NB_F64)
        return run_sym<SymF64>(sh, n, x, m, eps, G, acc, ws, ws_bytes, stream, kick_v, kick_h,
                               pot, drift_x, drift_dt);
    return hipErrorInvalidValue;
}

}  // namespace nb
