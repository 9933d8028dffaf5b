// Symmetric (third-law) form of the fused adjoint pair pass for the
// tile-compensated, plain FP32 and FP64 policies, on gfx950.
//
// With d = x_j - x_i, s = |d|^2 + eps^2, T(d) = s^-3/2 I - 3 s^-5/2 d d^T and
// u = m_i lam_j - m_j lam_i, the pair (i, j) adds
//   to i:  m_j s^-3/2 d,   T(d) u,    s^-3/2 (lam_j . d)
//   to j: -m_i s^-3/2 d,  -T(d) u,   -s^-3/2 (lam_i . d)
// (T is even in d and u is odd under the swap), so one reciprocal square
// root, one T(d) u and one s^-3/2 serve both ends: 42 VALU + 1 rsqrt per
// pair (d . u comes from the two dot products with lam_i and lam_j, which
// the mass adjoints need anyway, and the factor -3 of T with the masses),
// i.e. 21 VALU + 1/2 rsqrt per interaction against 34 + 1 one-sided.
// The blocking, the work items (block pairs I <= J), the origin of the pair
// arithmetic (tile-compensated policy: the centroid of block I), the
// source-side sums carried through the lanes and the fixed-order partials
// are those of the symmetric force pass, with seven quantities instead of
// three:
// a (3), J^T lam (3) and the mass-adjoint sum (1); the partials are in the
// pair type (FP32; FP64 for the FP64 policy). The items run in bands of
// block rows (SymLayout); after each band a fold kernel adds its partials
// in slot order to FP64 running sums and applies the adjoint epilogue of the
// reverse walk to the particles it completes, in the storage type as the
// one-sided pass's epilogue does.
#include "adjoint_sym_pairs.h"

namespace nb {

namespace {

using asym::ASymArgs;
using asym::NQ;
using asym::QRange;

// The fold of one band, as the symmetric force pass.
template <class Pol>
struct ASymFinishArgs {
    using pos_t = typename Pol::pos_t;
    const typename Pol::calc_t* part;
    SymBandView band;
    double* run;  // [NQF][n] running sums between bands, or nullptr
    int first;
    int n, nb;
    double G, c, h;
    int update_state;
    pos_t *ax, *ay, *az;
    pos_t *vx, *vy, *vz;
    pos_t *gx, *gy, *gz;
    double* gm;
    pos_t *rx, *ry, *rz;     // x of the next step's reverse drift, or nullptr
    pos_t *rlx, *rly, *rlz;  // lam_v written by that drift
    double dt;
};

// Slot-ordered FP64 sum of the partials, then the reverse-walk epilogue:
//   lam_x += c G J^T lam;  lam_m += c (-G) G^T-sum;
//   if update_state (F): acc = G a_sum; v <- v - h acc.
template <class Pol, bool F>
__global__ __launch_bounds__(256) void adjoint_sym_finish_kernel(ASymFinishArgs<Pol> a) {
    using pos_t = typename Pol::pos_t;
    constexpr int Q0 = QRange<F>::lo, NQF = QRange<F>::n;
    const SymBandView& b = a.band;
    const int i = b.base + blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    double q[NQ] = {0, 0, 0, 0, 0, 0, 0};
    if (!a.first) {
#pragma unroll
        for (int c = Q0; c < NQ; ++c) q[c] = a.run[(size_t)(c - Q0) * a.n + i];
    }
    // slots I0 .. I1-1 (region A): eight slots' loads in flight together,
    // the adds in slot order
#pragma unroll 8
    for (int k = b.I0; k < b.I1; ++k) {
#pragma unroll
        for (int c = Q0; c < NQ; ++c) q[c] += double(a.part[b.offset(k, c - Q0, i)]);
    }
    if (i >= b.base + b.nbp) {  // a later band adds this particle's next slots
#pragma unroll
        for (int c = Q0; c < NQ; ++c) a.run[(size_t)(c - Q0) * a.n + i] = q[c];
        return;
    }
    // the band's own particles: slots I1 .. nb-1 (region B), then finish
#pragma unroll 8
    for (int k = b.I1; k < a.nb; ++k) {
#pragma unroll
        for (int c = Q0; c < NQ; ++c) q[c] += double(a.part[b.offset(k, c - Q0, i)]);
    }
    const double G = a.G, c = a.c;
    a.gx[i] = pos_t(double(a.gx[i]) + c * (G * q[3]));
    a.gy[i] = pos_t(double(a.gy[i]) + c * (G * q[4]));
    a.gz[i] = pos_t(double(a.gz[i]) + c * (G * q[5]));
    a.gm[i] = a.gm[i] + c * (-G * q[6]);
    if (F) {
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

}  // namespace

bool adjoint_sym_shape_supported(int prec, const SymShape& s) {
    if (prec != NB_MIX_TILEC && prec != NB_F32 && prec != NB_F64) return false;
    // FP64 in 16-wave workgroups would spill (at most 128 VGPRs a lane there)
    const bool w16 = prec != NB_F64;
    return (s.ipl == 2 && (s.waves == 2 || s.waves == 4 || s.waves == 8 || (w16 && s.waves == 16))) ||
           (s.ipl == 1 && (s.waves == 4 || s.waves == 8)) ||
           (s.ipl == 4 && (s.waves == 2 || s.waves == 4 || s.waves == 8));
}

SymLayout adjoint_sym_layout(int prec, const SymShape& s, int64_t n, bool force_sums) {
    const int64_t bi = (int64_t)s.waves * 64 * s.ipl;
    return SymLayout{n, bi, (int)((n + bi - 1) / bi), force_sums ? QRange<true>::n : QRange<false>::n,
                     prec == NB_F64 ? sizeof(double) : sizeof(float), sizeof(double)};
}

SymShape choose_adjoint_sym_shape(int prec, int64_t n) {
    // Measured on MI355X with the tuner (tune.py; a walked-back step, the
    // pass with the force sums, and the entry pass without them; the run
    // these figures come from is in profiles/launch_shape_tuning.md):
    //  * below 163840 particles two sinks per lane -- the seven running sums
    //    per sink, each an FP32 group sum folded into FP64, take ~126 VGPRs
    //    -- in blocks of at most n/64 (256 or 512 particles; 65536: 4 waves x
    //    2, 2.33 ms, within 1 % of the fastest shape; 131072: the entry pass
    //    6.55 ms against 6.70 for the best shape with four sinks, the
    //    walked-back pass 8.96 against 8.57);
    //  * from 163840 four sinks per lane with FP32 block sums on the sink
    //    side (158 VGPRs with the force sums, 3 waves per SIMD; 159 and 3
    //    waves without them, as scheduled in their own translation unit) in
    //    4-wave blocks of 1024 at every n (163840: 10.39 / 13.20 ms against
    //    10.50 / 14.06 for 4 x 2, entry / walked-back pass; 196608: 14.74 /
    //    18.77 against 15.17 / 19.95):
    //    half the LDS reads and source-side rotations per pair -- 2^20: 542
    //    ms against 561 for 8 waves x 2; 2^21: 2165 ms against 2406 for 8
    //    waves x 4 (blocks of 2048: half the partials, but with 158 VGPRs a
    //    CU holds one eight-wave workgroup, two waves per SIMD, against three
    //    four-wave ones). The partials (nb * 7 * n floats, 30 GB at 2^20) are
    //    written and read back in bands of the workspace (SymLayout), so the
    //    pass serves every n up to 2^28 in bounded memory.
    // Below 12288 particles the one-sided kernel is faster (measured, with the
    // finishing kernel's loads overlapped: one-sided 31 % faster at 8192;
    // symmetric 12 % faster at 12288, 21 % at 24576).
    // The plain FP32 policy takes the same shapes (the tuner's fastest or
    // within 5 % of it for either pass: 65536 4 x 2, 1.59 / 1.94 ms for
    // entry / walked-back pass against 2.55 / 2.91 one-sided; 2^20 4 x 4,
    // 399 / 464 ms against 631 / 708). FP64 (two FP32 registers a value)
    // takes the fastest shape of the sweep at each size: 2 x 2 below 24576
    // (16384: 0.275 / 0.343 ms against 0.349 / 0.370 one-sided), 4 x 2 below
    // 49152 (24576: 0.530 / 0.663; 32768: 0.899 / 1.109, within 2.3 % of the
    // fastest), 2 x 4 below 98304 (65536: 3.03 / 3.93 against 4.92 / 5.35),
    // 4 x 4 from there (131072: 12.47 / 15.39; 262144: 45.8 / 57.2 against
    // 78.2 / 84.8; 2^20: 733 / 915 against 1241 / 1368).
    if ((prec != NB_MIX_TILEC && prec != NB_F32 && prec != NB_F64) || n < 48 * 256 ||
        n > (int64_t(1) << 28))
        return SymShape{0, 0};
    if (prec == NB_F64) {
        if (n < 24576) return SymShape{2, 2};  // 256
        if (n < 49152) return SymShape{4, 2};  // 512
        if (n < 98304) return SymShape{2, 4};  // 512
        return SymShape{4, 4};                 // 1024
    }
    auto bi = [](const SymShape& c) { return (int64_t)c.waves * 64 * c.ipl; };
    if (n < 163840) {
        static const SymShape small[] = {{2, 2}, {4, 2}};  // 256, 512
        return (bi(small[1]) <= n / 64) ? small[1] : small[0];
    }
    return SymShape{4, 4};  // 1024
}

namespace {

// One band's pair pass in shape sh; F: with the force sums.
template <class Pol, bool F>
hipError_t launch_pairs_shape(const SymShape& sh, const asym::ASymArgs<Pol>& a,
                              hipStream_t stream) {
    if constexpr (!F) {
        return asym::launch_pairs_entry(sh, a, stream);  // built with its own schedule
    } else {
#define NB_ASYM_CASE(WV, KV) \
    if (sh.waves == WV && sh.ipl == KV) return asym::launch_pairs<Pol, WV, KV, F>(a, stream);
        NB_ASYM_CASE(2, 2) NB_ASYM_CASE(4, 2) NB_ASYM_CASE(8, 2)
        NB_ASYM_CASE(4, 1) NB_ASYM_CASE(8, 1) NB_ASYM_CASE(2, 4) NB_ASYM_CASE(4, 4)
        NB_ASYM_CASE(8, 4)
        if constexpr (!std::is_same<typename Pol::calc_t, double>::value) {
            NB_ASYM_CASE(16, 2)
        }
#undef NB_ASYM_CASE
        return hipErrorInvalidValue;
    }
}

template <class Pol>
hipError_t launch_adjoint_sym_pol(int prec, const SymShape& sh, int64_t n, const void* x,
                                  const void* m, const void* lam_v, double eps, double G,
                                  double c, bool update_state, double h, void* acc, void* v,
                                  void* lam_x, double* lam_m, void* ws, size_t ws_bytes,
                                  hipStream_t stream, void* drift_x, double drift_dt) {
    using pos_t = typename Pol::pos_t;
    using mass_t = typename Pol::mass_t;
    using calc_t = typename Pol::calc_t;
    // the layout of this pass: seven partial rows with the force sums, four
    // without (the workspace is sized for seven)
    const SymLayout L = adjoint_sym_layout(prec, sh, n, update_state);
    const SymPlan plan = sym_plan(L, ws_bytes, sh.waves * 64);
    if (!plan.valid) return hipErrorInvalidValue;
    double* run = plan.one ? nullptr : static_cast<double*>(ws);
    calc_t* parts = reinterpret_cast<calc_t*>(static_cast<char*>(ws) + plan.parts);
    const size_t budget = plan.budget;

    asym::ASymArgs<Pol> a{};
    const pos_t* px = static_cast<const pos_t*>(x);
    const pos_t* pl = static_cast<const pos_t*>(lam_v);
    a.x = px;
    a.y = px + n;
    a.z = px + 2 * n;
    a.m = static_cast<const mass_t*>(m);
    a.lx = pl;
    a.ly = pl + n;
    a.lz = pl + 2 * n;
    a.n = (int)n;
    a.nb = L.nb;
    a.eps2 = calc_t(eps) * calc_t(eps);
    ASymFinishArgs<Pol> f{};
    f.run = run;
    f.n = a.n;
    f.G = G;
    f.c = c;
    f.h = h;
    f.update_state = update_state ? 1 : 0;  // also selects the kernels' force accumulation
    pos_t* pa = static_cast<pos_t*>(acc);
    pos_t* pv = static_cast<pos_t*>(v);
    pos_t* pg = static_cast<pos_t*>(lam_x);
    f.ax = pa; f.ay = pa + n; f.az = pa + 2 * n;
    f.vx = pv; f.vy = pv + n; f.vz = pv + 2 * n;
    f.gx = pg; f.gy = pg + n; f.gz = pg + 2 * n;
    f.gm = lam_m;
    if (drift_x) {  // each fold finishes particles after every read of their x and lam_v
        pos_t* prx = static_cast<pos_t*>(drift_x);
        pos_t* prl = static_cast<pos_t*>(const_cast<void*>(lam_v));
        f.rx = prx; f.ry = prx + n; f.rz = prx + 2 * n;
        f.rlx = prl; f.rly = prl + n; f.rlz = prl + 2 * n;
        f.dt = drift_dt;
    }
    a.part = parts;
    f.part = parts;
    f.nb = L.nb;
    for (int I0 = 0; I0 < L.nb;) {
        const int I1 = sym_band_end(L, I0, budget, sh.waves * 64);
        a.band = f.band = sym_band_view(L, I0, I1);
        hipError_t e = update_state ? launch_pairs_shape<Pol, true>(sh, a, stream)
                                    : launch_pairs_shape<Pol, false>(sh, a, stream);
        if (e != hipSuccess) return e;
        f.first = I0 == 0;
        const dim3 fg((unsigned)((a.band.np + 255) / 256));
        if (update_state)
            hipLaunchKernelGGL((adjoint_sym_finish_kernel<Pol, true>), fg, dim3(256), 0, stream, f);
        else
            hipLaunchKernelGGL((adjoint_sym_finish_kernel<Pol, false>), fg, dim3(256), 0, stream, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        I0 = I1;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_adjoint_sym(int prec, const SymShape& sh, int64_t n, const void* x,
                              const void* m, const void* lam_v, double eps, double G, double c,
                              bool update_state, double h, void* acc, void* v, void* lam_x,
                              double* lam_m, void* ws, size_t ws_bytes, hipStream_t stream,
                              void* drift_x, double drift_dt, bool* drifted) {
    if (drifted) *drifted = false;
    if ((int64_t)sh.waves * sh.ipl == 0) return hipErrorInvalidValue;
    hipError_t e = hipErrorInvalidValue;
    switch (prec) {
    case NB_MIX_TILEC:
        e = launch_adjoint_sym_pol<PolMixTileC>(prec, sh, n, x, m, lam_v, eps, G, c, update_state,
                                                h, acc, v, lam_x, lam_m, ws, ws_bytes, stream,
                                                drift_x, drift_dt);
        break;
    case NB_F32:
        e = launch_adjoint_sym_pol<PolF32>(prec, sh, n, x, m, lam_v, eps, G, c, update_state, h,
                                           acc, v, lam_x, lam_m, ws, ws_bytes, stream, drift_x,
                                           drift_dt);
        break;
    case NB_F64:
        e = launch_adjoint_sym_pol<PolF64>(prec, sh, n, x, m, lam_v, eps, G, c, update_state, h,
                                           acc, v, lam_x, lam_m, ws, ws_bytes, stream, drift_x,
                                           drift_dt);
        break;
    default:
        break;
    }
    if (e == hipSuccess && drifted) *drifted = drift_x != nullptr;
    return e;
}

}  // namespace nb
