// Private header of libnbody: precision traits, per-sink accumulators and
// the reciprocal square roots shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "nbody.h"

namespace nb {

// Fused multiply-add in the operands' own type (__builtin_fma alone would
// promote float operands to double).
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Reciprocal square roots.
//
// FP32: the hardware v_rsq_f32 (about 1 ulp). The paper notes that a fast
// approximate reciprocal square root is what makes this kernel fast on every
// GPU it measured (section "N-body simulation").
// FP64: v_rsq_f64 as a first guess y (about 24 correct bits), then one
// third-order correction: with e = 1 - s y^2 (formed with an FMA),
// s^-1/2 = y (1 - e)^-1/2 = y (1 + e/2 + 3e^2/8 + 5e^3/16 + ...), and the
// series cut after e^2 leaves 5e^3/16 ~ 2^-70: five FP64 operations instead
// of eight for two Newton-Raphson steps, with the same ~1 ulp result.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rsqrt_pair(float s) { return __builtin_amdgcn_rsqf(s); }

__device__ __forceinline__ double rsqrt_pair(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    const double e = __builtin_fma(-s * y, y, 1.0);
    const double p = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, p, y);
}

// ---------------------------------------------------------------------------
// Per-sink running sums (one component each).
// ---------------------------------------------------------------------------

// Plain running sum in the pair-arithmetic type T: s = fma(d, w, s), the
// listing's accumulation.
template <typename T>
struct SumPlain {
    T s;
    __device__ __forceinline__ void init() { s = T(0); }
    __device__ __forceinline__ void add_fma(T d, T w) { s = fmat(d, w, s); }
    __device__ __forceinline__ void add(T t) { s += t; }
    __device__ __forceinline__ void tile_end() {}
    __device__ __forceinline__ double total() const { return double(s); }
};

// Kahan-compensated FP32 running sum. The term d*w - c is formed with one
// FMA, then t = s + y; c = (t - s) - y recovers the rounding error of the
// addition (exact when |s| >= |y|) and feeds it back into the next term.
struct SumKahan {
    float s, c;
    __device__ __forceinline__ void init() { s = 0.f; c = 0.f; }
    __device__ __forceinline__ void add_y(float y) {
        float t = s + y;
        // keep the compensation: no reassociation (the library is compiled without fast-math)
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ void add_fma(float d, float w) { add_y(__builtin_fmaf(d, w, -c)); }
    __device__ __forceinline__ void add(float t) { add_y(t - c); }
    __device__ __forceinline__ void tile_end() {}
    __device__ __forceinline__ double total() const { return double(s) - double(c); }
};

// FP32 terms summed in FP64: the exact product of the FP32 factors is added
// with an FP64 FMA.
struct SumWide {
    double s;
    __device__ __forceinline__ void init() { s = 0.0; }
    __device__ __forceinline__ void add_fma(float d, float w) {
        s = __builtin_fma(double(d), double(w), s);
    }
    __device__ __forceinline__ void add(float t) { s += double(t); }
    __device__ __forceinline__ void tile_end() {}
    __device__ __forceinline__ double total() const { return s; }
};

// FP32 running sum over one j-tile, folded into an FP64 total at the end of
// every tile: FP32 cost per pair, and the FP32 error grows only with the tile
// length instead of with N.
struct SumTile {
    float p;
    double s;
    __device__ __forceinline__ void init() { p = 0.f; s = 0.0; }
    __device__ __forceinline__ void add_fma(float d, float w) { p = __builtin_fmaf(d, w, p); }
    __device__ __forceinline__ void add(float t) { p += t; }
    __device__ __forceinline__ void tile_end() { s += double(p); p = 0.f; }
    __device__ __forceinline__ double total() const { return s + double(p); }
};

// Lane l receives the value of lane (l + 1) mod 64, through the LDS
// crossbar (ds_bpermute): measured 14 % faster for the force pass and 10 %
// for the adjoint than the same rotation on the vector ALU (DPP wave_rol:1),
// whose moves cost about four VALU issue slots each and sit in the
// accumulation chains; the crossbar is otherwise idle here. The symmetric
// passes carry their source-side sums through the lanes with it.
__device__ __forceinline__ float from_next_lane(float v) {
    const int src = ((__lane_id() + 1) & 63) << 2;  // byte address of the source lane
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
}

// The same for a double: its two 32-bit halves travel separately.
__device__ __forceinline__ double from_next_lane(double v) {
    const int src = ((__lane_id() + 1) & 63) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Origin of the FP32 pair arithmetic in the mixed policies.
//
// There positions are FP64 and the pair arithmetic FP32. Rounding x itself
// to FP32 would give the separation d = x_j - x_i an absolute error of up to
// 2^-24 (|x_i| + |x_j|): relative error 2^-24 |x| / |d|, growing with the
// distance from the coordinate origin. Instead every workgroup subtracts,
// in FP64, the centroid o of its own sinks (one contiguous index range)
// from those sinks and from every source it stages, and rounds x - o: the
// error of d is then at most 2^-24 (|x_i - o| + |x_j - o|), whatever the
// position of the system, and the same d serves both ends of a pair in the
// symmetric passes. The centroid is a fixed-order FP64 reduction (xor
// butterfly within each wave -- every lane ends with bitwise the same sum --
// then the wave sums in wave order), so results stay reproducible.
//
// s*: this thread's FP64 sum over its valid sinks; count: valid sinks of the
// workgroup (>= 1); lds: NW x 3 doubles of shared memory. Contains a
// workgroup barrier: every thread of the workgroup must call it.
// ---------------------------------------------------------------------------
// A value that every lane of the wave holds, moved to a scalar register.
__device__ __forceinline__ double wave_uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

template <int NW>
__device__ __forceinline__ void sink_block_origin(double sx, double sy, double sz, int count,
                                                  double (*lds)[3], double& ox, double& oy,
                                                  double& oz) {
#pragma unroll
    for (int mask = 32; mask >= 1; mask >>= 1) {
        sx += __shfl_xor(sx, mask, 64);
        sy += __shfl_xor(sy, mask, 64);
        sz += __shfl_xor(sz, mask, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        lds[w][0] = sx;
        lds[w][1] = sy;
        lds[w][2] = sz;
    }
    __syncthreads();
    double tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
        tx += lds[v][0];
        ty += lds[v][1];
        tz += lds[v][2];
    }
    // every lane holds bitwise the same origin: keep it in scalar registers
    // (the pair loops need every vector register they can get)
    const double c = double(count);
    ox = wave_uniform(tx / c);
    oy = wave_uniform(ty / c);
    oz = wave_uniform(tz / c);
}

// ---------------------------------------------------------------------------
// Precision traits: storage types and the pair-arithmetic type.
// ---------------------------------------------------------------------------
template <typename Pos, typename Mass, typename Calc, typename Sum>
struct Policy {
    using pos_t = Pos;    // positions, velocities, accelerations, adjoints
    using mass_t = Mass;  // masses
    using calc_t = Calc;  // pair arithmetic
    using sum_t = Sum;    // per-sink running sum
    // FP64 positions, FP32 pair arithmetic: positions are taken relative to
    // the sink block's centroid before they are rounded (sink_block_origin)
    static constexpr bool origin =
        std::is_same<Pos, double>::value && std::is_same<Calc, float>::value;
};

// A stored coordinate as the pair arithmetic takes it: relative to the
// origin o in FP64, then rounded, where the policy has an origin; else the
// coordinate converted as it is (o is then ignored; it is 0).
template <class Pol>
__device__ __forceinline__ typename Pol::calc_t pair_coord(typename Pol::pos_t x, double o) {
    using calc_t = typename Pol::calc_t;
    if constexpr (Pol::origin)
        return calc_t(double(x) - o);
    else
        return calc_t(x);
}

using PolF64 = Policy<double, double, double, SumPlain<double>>;
using PolF32 = Policy<float, float, float, SumPlain<float>>;
using PolMixAcc32 = Policy<double, float, float, SumPlain<float>>;
using PolMixKahan = Policy<double, float, float, SumKahan>;
using PolMixAcc64 = Policy<double, float, float, SumWide>;
using PolMixTileC = Policy<double, float, float, SumTile>;

// 4-vector LDS record of the pair-arithmetic type.
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

inline size_t pos_size(int prec) { return prec == NB_F32 ? 4 : 8; }
inline size_t mass_size(int prec) { return (prec == NB_F64) ? 8 : 4; }

// Calls f(PolicyTag{}) with the policy of `prec`; returns false if unknown.
template <typename F>
inline bool dispatch_prec(int prec, F&& f) {
    switch (prec) {
    case NB_F64: f(PolF64{}); return true;
    case NB_F32: f(PolF32{}); return true;
    case NB_MIX_ACC32: f(PolMixAcc32{}); return true;
    case NB_MIX_KAHAN: f(PolMixKahan{}); return true;
    case NB_MIX_ACC64: f(PolMixAcc64{}); return true;
    case NB_MIX_TILEC: f(PolMixTileC{}); return true;
    default: return false;
    }
}

// ---------------------------------------------------------------------------
// Host-side launch shapes and the functions each kernel file provides.
// ---------------------------------------------------------------------------
struct Shape {
    int ipl;    // sinks per lane
    int block;  // threads per workgroup = j-tile length
    int split;  // j-ranges per sink
};

// Library choice of shape for ni sinks, nj sources.
Shape choose_force_shape(int prec, int64_t ni, int64_t nj);
Shape choose_adjoint_shape(int prec, int64_t n);
// Shapes the one-sided force / adjoint kernels are built for.
bool shape_supported(const Shape& s);
bool adjoint_shape_supported(const Shape& s);

// Workspace bytes of the split partials of a force / adjoint launch.
size_t force_partials_bytes(const Shape& s, int64_t ni);
// Bound of the one-sided force partials over all ni, nj <= n.
size_t force_partials_bound(int64_t n);
size_t adjoint_partials_bytes(const Shape& s, int64_t n);

// Force: acc (and pot) of ni sinks. self_set: xi and xj are the same set.
// kick_v (optional, 3 ni pos elements): also apply v <- v + kick_h * acc in
// the epilogue, with acc as stored (the leapfrog's closing half-kick).
// drift_x (optional, with kick_v, self set): then also the next step's
// kick and drift, v <- v + kick_h * acc; x <- x + drift_dt * v, when the
// pass has a finishing kernel that runs after every read of x; *drifted
// (if given) tells whether it did.
hipError_t launch_force(int prec, const Shape& shape, int64_t ni, const void* xi,
                        int64_t nj, const void* xj, const void* mj, double eps,
                        double G, bool self_set, void* acc, void* pot, void* ws,
                        hipStream_t stream, void* kick_v = nullptr, double kick_h = 0.0,
                        void* drift_x = nullptr, double drift_dt = 0.0,
                        bool* drifted = nullptr);

// Symmetric (third-law) force pass of one set on itself, NB_MIX_TILEC, NB_F32
// and NB_F64: blocks of waves*64*ipl particles; waves == 0 means "not used". pot:
// the pass also computes the potential (four partial quantities, not three).
struct SymShape {
    int waves;  // wavefronts per workgroup
    int ipl;    // sinks per lane
};

// ---------------------------------------------------------------------------
// Bands of the symmetric passes (host side).
//
// A symmetric pass over nb blocks has one work item per block pair (I, J),
// I <= J, and every particle of block P receives one partial in each slot
// k = 0 .. nb-1 (the source side of item (k, P) for k < P, item (P, P), the
// sink side of item (P, k) for k > P), which a finishing kernel adds in slot
// order. The items are launched in bands of consecutive rows I0 <= I < I1.
// A band writes, for every particle from block I0 on, its slots I0 .. I1-1
// (region A) and, for the particles of its own blocks, their slots I1 ..
// nb-1 (region B: the sink sides of items (I, J), J >= I1); a fold kernel
// then adds them, in slot order, to a running sum per particle kept between
// bands in the finishing type, and finishes the band's own particles, whose
// slots are then complete and which no later band reads (later bands touch
// blocks >= I1 only). The sums are therefore bitwise those of one launch
// over every item, while the scratch is one band's partials plus the
// running sums. With a workspace that holds every partial the pass is one
// band (no running sums).
// ---------------------------------------------------------------------------
struct SymLayout {
    int64_t n;    // particles
    int64_t bi;   // particles per block
    int nb;       // blocks
    int nq;       // partial quantities per particle
    size_t elem;  // bytes of a partial
    size_t fin;   // bytes of a running-sum element
};

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of the partials of band [I0, I1): region A then region B.
inline size_t sym_band_bytes(const SymLayout& L, int I0, int I1) {
    const int64_t base = (int64_t)I0 * L.bi;
    const int64_t np = L.n - base;
    const int64_t nbp = std::min<int64_t>(L.n, (int64_t)I1 * L.bi) - base;
    return ((size_t)(I1 - I0) * (size_t)np + (size_t)(L.nb - I1) * (size_t)nbp) *
           (size_t)L.nq * L.elem;
}
// Every partial at once (one band).
inline size_t sym_full_bytes(const SymLayout& L) { return sym_band_bytes(L, 0, L.nb); }
// The running sums, placed at the start of a banded workspace.
inline size_t sym_run_bytes(const SymLayout& L) {
    return align256((size_t)L.nq * (size_t)L.n * L.fin);
}
// The least workspace the pass runs in: every partial at once, or one row
// per band (the first row needs the most) and the running sums, whichever is
// less (where a single band would launch too many threads, the second: it is
// then far below the first).
inline size_t sym_min_bytes(const SymLayout& L) {
    return std::min(sym_full_bytes(L), sym_run_bytes(L) + sym_band_bytes(L, 0, 1));
}
// Workspace the library asks for: every partial up to kSymBandBudget, else
// bands of about that much.
constexpr size_t kSymBandBudget = size_t(4) << 30;
inline size_t sym_default_bytes(const SymLayout& L) {
    const size_t full = sym_full_bytes(L);
    if (full <= kSymBandBudget) return full;
    return sym_run_bytes(L) + std::max(kSymBandBudget, sym_band_bytes(L, 0, 1));
}
// How a pass uses a workspace of ws bytes: one band over every item when
// the workspace holds every partial and the items launch in one grid (fewer
// than 2^31 threads of nt per item); else the running sums at the start of
// the workspace and bands of at most `budget` bytes of partials after them.
// valid = false: the workspace is below sym_min_bytes.
struct SymPlan {
    bool valid, one;
    size_t parts;   // offset of the partials in the workspace
    size_t budget;  // bytes of partials per band
};
inline int64_t sym_band_items(const SymLayout& L, int I0, int I1);
inline SymPlan sym_plan(const SymLayout& L, size_t ws, int nt) {
    const size_t full = sym_full_bytes(L);
    if (ws >= full && sym_band_items(L, 0, L.nb) < (int64_t(1) << 31) / nt)
        return SymPlan{true, true, 0, full};
    const size_t run = sym_run_bytes(L);
    const bool valid = ws >= run + sym_band_bytes(L, 0, 1);
    return SymPlan{valid, false, run, valid ? ws - run : 0};
}

// Work items (block pairs) of band [I0, I1).
inline int64_t sym_band_items(const SymLayout& L, int I0, int I1) {
    const int64_t R = I1 - I0;
    return R * (R + 1) / 2 + R * (L.nb - I1);
}
// Last row (exclusive) of the band that starts at I0, fits `budget` bytes of
// partials and launches fewer than 2^31 threads (nt per item): the band
// grows while both hold (both grow with I1), and is at least one row (at
// most nb items of <= 1024 threads).
inline int sym_band_end(const SymLayout& L, int I0, size_t budget, int nt) {
    const int64_t max_items = (int64_t(1) << 31) / nt - 1;
    int lo = I0 + 1, hi = L.nb;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (sym_band_bytes(L, I0, mid) <= budget && sym_band_items(L, I0, mid) <= max_items)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Work item t of the band [I0, I1) -> block pair (I, J), I <= J: first the
// triangle of pairs inside the band (J < I1), then the rectangle of rows
// I0 .. I1-1 against the blocks J >= I1; in both, items ordered by J, then
// I, so that consecutive workgroups share their source block.
__host__ __device__ inline void band_item(int64_t t, int I0, int I1, int& I, int& J) {
    const int R = I1 - I0;
    const int64_t tri = (int64_t)R * (R + 1) / 2;
    if (t < tri) {
        int j = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)j * (j + 1) / 2 > t) --j;
        while ((int64_t)(j + 1) * (j + 2) / 2 <= t) ++j;
        I = I0 + (int)(t - (int64_t)j * (j + 1) / 2);
        J = I0 + j;
    } else {
        const int64_t u = t - tri;
        J = I1 + (int)(u / R);
        I = I0 + (int)(u % R);
    }
}

// Where one band's partials live: element offsets from the start of its
// partials, region A (slots I0 .. I1-1 of every particle from `base` on,
// rows of np) followed by region B (slots I1 .. nb-1 of the band's own nbp
// particles, rows of nbp); quantity c of nq.
struct SymBandView {
    int I0, I1;  // the band's rows
    int base;    // first particle of block I0
    int np;      // particles base .. n-1
    int nbp;     // particles of blocks I0 .. I1-1
    int nq;      // partial quantities per particle and slot
    // slot k (I0 <= k < nb) of particle p (p < base + nbp when k >= I1)
    __host__ __device__ size_t offset(int k, int c, int p) const {
        return k < I1 ? ((size_t)(k - I0) * nq + c) * np + (size_t)(p - base)
                      : (size_t)(I1 - I0) * nq * np + ((size_t)(k - I1) * nq + c) * nbp +
                            (size_t)(p - base);
    }
};
inline SymBandView sym_band_view(const SymLayout& L, int I0, int I1) {
    const int base = (int)(I0 * L.bi);
    return SymBandView{I0, I1, base, (int)(L.n - base),
                       (int)(std::min<int64_t>(L.n, I1 * L.bi) - base), L.nq};
}

SymShape choose_sym_shape(int prec, int64_t n, bool pot = false);
// Shapes the symmetric force pass is built for (and policies that have it).
bool sym_shape_supported(int prec, const SymShape& s);
// The band layout of the symmetric force pass.
SymLayout sym_layout(int prec, const SymShape& s, int64_t n, bool pot = false);
// acc = a(x) (and with kick_v, v <- v + kick_h * acc; with pot, the
// potential with the j = i term removed); ws holds ws_bytes >=
// sym_min_bytes(sym_layout(prec, sh, n, pot != nullptr)) bytes, used in
// bands as above (one band when it holds every partial).
// drift_x / drift_dt / drifted: as launch_force (each finishing kernel runs
// after every read of its particles' positions, so the drift is always taken
// when asked for).
hipError_t launch_force_sym(int prec, const SymShape& sh, int64_t n, const void* x,
                            const void* m, double eps, double G, void* acc, void* ws,
                            size_t ws_bytes, hipStream_t stream, void* kick_v = nullptr,
                            double kick_h = 0.0, void* pot = nullptr, void* drift_x = nullptr,
                            double drift_dt = 0.0, bool* drifted = nullptr);

// Fused adjoint pair pass at x with adjoint lam_v: computes a(x), J^T lam_v,
// G^T lam_v and applies the epilogue
//   lam_x += c J^T lam_v;  lam_m += c G^T lam_v;
//   if update_state: acc = a(x); v = v - h acc.
// drift_x (optional): then also the next step's reverse drift,
//   lam_v += drift_dt lam_x; v -= h acc; x -= drift_dt v,
// where the pass has a finishing kernel that runs after every read of x and
// lam_v (*drifted, if given, tells whether it did).
hipError_t launch_adjoint(int prec, const Shape& shape, int64_t n, const void* x,
                          const void* m, const void* lam_v, double eps, double G,
                          double c, bool update_state, double h, void* acc, void* v,
                          void* lam_x, double* lam_m, void* ws, hipStream_t stream,
                          void* drift_x = nullptr, double drift_dt = 0.0,
                          bool* drifted = nullptr);

// Symmetric form of the fused adjoint pass (NB_MIX_TILEC, NB_F32, NB_F64),
// same contract as launch_adjoint; ws holds ws_bytes >= sym_min_bytes(
// adjoint_sym_layout(prec, sh, n, true)) bytes, used in bands as the force
// pass. force_sums: the layout of a pass that also sums a(x) (seven
// quantities; four without), which update_state asks for.
SymShape choose_adjoint_sym_shape(int prec, int64_t n);
bool adjoint_sym_shape_supported(int prec, const SymShape& s);
SymLayout adjoint_sym_layout(int prec, const SymShape& s, int64_t n, bool force_sums);
hipError_t launch_adjoint_sym(int prec, const SymShape& sh, int64_t n, const void* x, const void* m,
                              const void* lam_v, double eps, double G, double c,
                              bool update_state, double h, void* acc, void* v, void* lam_x,
                              double* lam_m, void* ws, size_t ws_bytes, hipStream_t stream,
                              void* drift_x = nullptr, double drift_dt = 0.0,
                              bool* drifted = nullptr);

// O(N) leapfrog kernels over the 3n components of a pos array.
hipError_t launch_kick_drift(int prec, int64_t n, void* x, void* v, const void* acc,
                             double h, double dt, hipStream_t stream);
// Reverse drift: lam_v += dt lam_x; v <- v - h acc; x <- x - dt v.
hipError_t launch_reverse_drift(int prec, int64_t n, void* x, void* v, const void* acc,
                                const void* lam_x, void* lam_v, double h, double dt,
                                hipStream_t stream);
// lam_v += dt lam_x only (before a checkpoint reload).
hipError_t launch_axpy_pos(int prec, int64_t n3, void* y, const void* xv, double a,
                           hipStream_t stream);

// One step of the 3-D diffusion stencil (FP32 grid, k fastest).
hipError_t launch_diffusion3d(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                              double dt, double kappa, const float* f, float* fn, hipStream_t stream);

// ---------------------------------------------------------------------------
// Entry-point plumbing shared by the ABI translation units.
// ---------------------------------------------------------------------------
// The pass nbody_accel runs for a call, once its arguments are checked.
struct AccelPlan {
    SymShape sym;   // the symmetric pass (sym.waves != 0), or
    Shape sh;       // the one-sided kernel in this shape
    bool self_set;
    size_t need;    // scratch bytes the pass needs at least
    size_t full;    // scratch bytes it uses at most (every partial at once)
};
// Checks the arguments of nbody_accel / nbody_accel_ex (not the workspace)
// and fills *plan; returns an nb_status.
int accel_plan(int64_t ni, const void* xi, int64_t nj, const void* xj, const void* mj,
               double eps, double G, int prec, void* acc, void* pot, const nb_launch* launch,
               AccelPlan* plan);
// Enqueues the planned pass with ws_bytes >= plan.need bytes of scratch at ws.
hipError_t accel_launch(const AccelPlan& p, int64_t ni, const void* xi, int64_t nj, const void* xj,
                        const void* mj, double eps, double G, int prec, void* acc, void* pot,
                        void* ws, size_t ws_bytes, hipStream_t s);
// NB_OK if a gfx950 device is current, else NB_ENODEV.
int check_device();
// NB_OK, or NB_EDEVICE after recording the HIP error for nbody_last_hip_error.
int hip_status(hipError_t e);

// FP64 diagnostics into out[13] (device).
size_t diag_workspace_bytes(int64_t n);
hipError_t launch_diag(int prec, int64_t n, const void* x, const void* v, const void* m,
                       double eps, double G, double* out, void* ws, hipStream_t stream);

}  // namespace nb
