// C ABI of libnbody (declared in include/nbody.h): argument checks, launch
// shapes, and the host loops of the leapfrog and of its reverse walk.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "common.h"
#include "diffusion3d.h"

namespace {

using namespace nb;

thread_local int g_last_hip_error = 0;

// ---- device-time profile (nbody_profile_begin / nbody_profile_end) --------
struct ProfRec {
    int kind;
    hipEvent_t a, b;
};
thread_local bool g_prof = false;
thread_local std::vector<ProfRec> g_recs;
thread_local std::vector<hipEvent_t> g_pool;

hipEvent_t pooled_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs f() (which enqueues work on s); while profiling, brackets it with events.
template <class F>
hipError_t timed(int kind, hipStream_t s, F&& f) {
    if (!g_prof) return f();
    hipEvent_t a = pooled_event(), b = pooled_event();
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = f();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    g_recs.push_back({kind, a, b});
    return e;
}

constexpr int64_t kMaxN = int64_t(1) << 30;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool valid_prec(int prec) { return prec >= NB_F64 && prec <= NB_MIX_TILEC; }

bool valid_eps(double eps, int prec) {
    if (!isfinite(eps) || !(eps > 0.0)) return false;
    // FP32 pair arithmetic needs eps^2 and eps^-3 to stay normal and finite
    if (prec != NB_F64 && eps < 0x1p-40) return false;
    if (prec == NB_F64 && eps < 1e-100) return false;
    return true;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

namespace nb {

// A gfx950 device must be current. The answer is cached per device id.
int check_device() {
    static std::atomic<int> cache[64];  // 0 unknown, 1 ok, 2 not gfx950
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return NB_ENODEV;
    }
    if (dev < 64 && cache[dev].load() == 1) return NB_OK;
    if (dev < 64 && cache[dev].load() == 2) return NB_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return NB_ENODEV;
    }
    const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev < 64) cache[dev].store(ok ? 1 : 2);
    return ok ? NB_OK : NB_ENODEV;
}

int hip_status(hipError_t e) {
    if (e == hipSuccess) return NB_OK;
    g_last_hip_error = (int)e;
    return NB_EDEVICE;
}

}  // namespace nb

namespace {

int check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return NB_OK;
    if (!ws || !aligned(ws, 256) || ws_bytes < need) return NB_EWORKSPACE;
    return NB_OK;
}

size_t accel_ws(const Shape& s, int64_t ni) {
    return s.split > 1 ? force_partials_bytes(s, ni) : 0;
}

hipError_t copy_state(void* dst, const void* src, size_t bytes, hipStream_t stream) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream);
}

// ---- instantiated leapfrog graphs (nbody_step with NB_GRAPH) ---------------
// A graph is recorded on a library-owned capture stream of the device (so the
// caller's stream may be the null stream), instantiated once per distinct
// argument set, and replayed with hipGraphLaunch on the caller's stream.
struct StepKey {
    int dev;
    int prec;
    unsigned flags;
    int64_t n, nsteps, ckpt_every;
    const void *x, *v, *m, *acc, *ckpt, *ws;
    size_t ws_bytes;
    double eps, G, dt;
};

struct GraphEntry {
    StepKey key;
    hipGraphExec_t exec;
    hipEvent_t done;  // recorded after the entry's latest launch
    uint64_t used;
};

constexpr size_t kGraphCacheMax = 16;
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
hipStream_t g_capture_stream[64] = {};

// Field by field: a copied key need not carry its padding bytes along.
bool same_key(const StepKey& a, const StepKey& b) {
    return a.dev == b.dev && a.prec == b.prec && a.flags == b.flags && a.n == b.n &&
           a.nsteps == b.nsteps && a.ckpt_every == b.ckpt_every && a.x == b.x && a.v == b.v &&
           a.m == b.m && a.acc == b.acc && a.ckpt == b.ckpt && a.ws == b.ws &&
           a.ws_bytes == b.ws_bytes && a.eps == b.eps && a.G == b.G && a.dt == b.dt;
}

// Waits for the entry's last launch, then frees it. Caller holds g_graph_mu.
hipError_t release_graph(GraphEntry& g) {
    hipError_t e = hipEventSynchronize(g.done);
    hipError_t e2 = hipGraphExecDestroy(g.exec);
    hipError_t e3 = hipEventDestroy(g.done);
    return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : e3);
}

// Replays the graph of `key` on s, recording it first with enqueue(q) on the
// capture stream q if it is not cached.
template <class F>
hipError_t graph_launch(const StepKey& key, hipStream_t s, F&& enqueue) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    GraphEntry* hit = nullptr;
    for (GraphEntry& g : g_graphs)
        if (same_key(g.key, key)) hit = &g;
    if (!hit) {
        if (key.dev < 0 || key.dev >= 64) return hipErrorInvalidDevice;
        hipError_t e = hipSuccess;
        if (g_graphs.size() >= kGraphCacheMax) {
            size_t lru = 0;
            for (size_t k = 1; k < g_graphs.size(); ++k)
                if (g_graphs[k].used < g_graphs[lru].used) lru = k;
            e = release_graph(g_graphs[lru]);
            g_graphs.erase(g_graphs.begin() + (ptrdiff_t)lru);
            if (e != hipSuccess) return e;
        }
        hipStream_t& q = g_capture_stream[key.dev];
        if (!q && (e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking)) != hipSuccess) {
            q = nullptr;
            return e;
        }
        if ((e = hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
        const hipError_t recorded = enqueue(q);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(q, &graph);
        if (recorded != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return recorded != hipSuccess ? recorded : e;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        hipEvent_t done = nullptr;
        if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) {
            (void)hipGraphExecDestroy(exec);
            return e;
        }
        g_graphs.push_back(GraphEntry{key, exec, done, 0});
        hit = &g_graphs.back();
    }
    hit->used = ++g_graph_clock;
    hipError_t e = hipGraphLaunch(hit->exec, s);
    if (e == hipSuccess) e = hipEventRecord(hit->done, s);
    return e;
}

// The symmetric shape a launch asks for: both fields given, or both 0 for
// the library's choice (which must then be the symmetric pass).
int sym_from_launch(const nb_launch& l, SymShape lib, SymShape* out) {
    if (l.split > 1) return NB_EUNSUPPORTED;
    if (l.block == 0 && l.i_per_lane == 0) {
        if (!lib.waves) return NB_EUNSUPPORTED;
        *out = lib;
        return NB_OK;
    }
    if (l.block <= 0 || l.block % 64 != 0) return NB_EUNSUPPORTED;
    *out = SymShape{l.block / 64, l.i_per_lane};
    return NB_OK;
}

// The pass and shape of a force call: the symmetric pass for one set on
// itself where the policy has one and no launch overrides it; else the
// one-sided kernel in the library's shape with the launch's fields.
int resolve_accel(int prec, int64_t ni, int64_t nj, bool self_set, bool pot,
                  const nb_launch* launch, SymShape* sym, Shape* sh) {
    *sym = (self_set && !launch) ? choose_sym_shape(prec, ni, pot) : SymShape{0, 0};
    *sh = choose_force_shape(prec, ni, nj);
    if (!launch) return NB_OK;
    if (launch->symmetric) {
        if (!self_set) return NB_EUNSUPPORTED;
        const int st = sym_from_launch(*launch, choose_sym_shape(prec, ni, pot), sym);
        if (st != NB_OK) return st;
        return sym_shape_supported(prec, *sym) ? NB_OK : NB_EUNSUPPORTED;
    }
    if (launch->i_per_lane) sh->ipl = launch->i_per_lane;
    if (launch->block) sh->block = launch->block;
    if (launch->split) sh->split = launch->split;
    return shape_supported(*sh) ? NB_OK : NB_EUNSUPPORTED;
}

// The same for the fused adjoint pass of n particles.
int resolve_adjoint(int prec, int64_t n, const nb_launch* launch, SymShape* sym, Shape* sh) {
    *sym = choose_adjoint_sym_shape(prec, n);
    *sh = choose_adjoint_shape(prec, n);
    if (!launch) return NB_OK;
    if (launch->symmetric) {
        const int st = sym_from_launch(*launch, *sym, sym);
        if (st != NB_OK) return st;
        return adjoint_sym_shape_supported(prec, *sym) ? NB_OK : NB_EUNSUPPORTED;
    }
    *sym = SymShape{0, 0};
    if (launch->i_per_lane) sh->ipl = launch->i_per_lane;
    if (launch->block) sh->block = launch->block;
    if (launch->split) sh->split = launch->split;
    return adjoint_shape_supported(*sh) ? NB_OK : NB_EUNSUPPORTED;
}

size_t adjoint_partials_need(int prec, const SymShape& sym, const Shape& sh, int64_t n, bool least) {
    if (sym.waves) {
        const SymLayout L = adjoint_sym_layout(prec, sym, n, true);
        return least ? sym_min_bytes(L) : sym_default_bytes(L);
    }
    return sh.split > 1 ? adjoint_partials_bytes(sh, n) : 0;
}

}  // namespace

namespace nb {

int accel_plan(int64_t ni, const void* xi, int64_t nj, const void* xj, const void* mj,
               double eps, double G, int prec, void* acc, void* pot, const nb_launch* launch,
               AccelPlan* plan) {
    if (!valid_prec(prec)) return NB_EUNSUPPORTED;
    if (ni < 1 || nj < 1 || ni > kMaxN || nj > kMaxN) return NB_EINVAL;
    if (!valid_eps(eps, prec) || !isfinite(G)) return NB_EINVAL;
    const size_t ps = pos_size(prec), ms = mass_size(prec);
    if (!xi || !xj || !mj || !acc) return NB_EINVAL;
    if (!aligned(xi, ps) || !aligned(xj, ps) || !aligned(mj, ms) || !aligned(acc, ps) ||
        (pot && !aligned(pot, ps)))
        return NB_EINVAL;
    const bool self_set = (xi == xj);
    if (self_set && ni != nj) return NB_EINVAL;
    const size_t acc_b = 3 * (size_t)ni * ps;
    if (overlaps(acc, acc_b, xi, 3 * (size_t)ni * ps) || overlaps(acc, acc_b, xj, 3 * (size_t)nj * ps) ||
        overlaps(acc, acc_b, mj, (size_t)nj * ms))
        return NB_EINVAL;
    if (pot && (overlaps(pot, (size_t)ni * ps, acc, acc_b) ||
                overlaps(pot, (size_t)ni * ps, xi, 3 * (size_t)ni * ps) ||
                overlaps(pot, (size_t)ni * ps, xj, 3 * (size_t)nj * ps) ||
                overlaps(pot, (size_t)ni * ps, mj, (size_t)nj * ms)))
        return NB_EINVAL;
    Shape sh;
    const int st = resolve_accel(prec, ni, nj, self_set, pot != nullptr, launch, &plan->sym, &sh);
    if (st != NB_OK) return st;
    plan->sh = sh;
    plan->self_set = self_set;
    if (plan->sym.waves) {
        const SymLayout L = sym_layout(prec, plan->sym, ni, pot != nullptr);
        plan->need = sym_min_bytes(L);
        plan->full = sym_full_bytes(L);
    } else {
        plan->need = plan->full = accel_ws(sh, ni);
    }
    return NB_OK;
}

}  // namespace nb

namespace {

// The scratch must not overlap any buffer of the call.
bool accel_ws_overlaps(const void* ws, size_t need, int64_t ni, const void* xi, int64_t nj,
                       const void* xj, const void* mj, int prec, const void* acc, const void* pot) {
    if (need == 0) return false;
    const size_t ps = pos_size(prec), ms = mass_size(prec);
    return overlaps(ws, need, xi, 3 * (size_t)ni * ps) || overlaps(ws, need, xj, 3 * (size_t)nj * ps) ||
           overlaps(ws, need, mj, (size_t)nj * ms) || overlaps(ws, need, acc, 3 * (size_t)ni * ps) ||
           overlaps(ws, need, pot, (size_t)ni * ps);
}

}  // namespace

namespace nb {

hipError_t accel_launch(const AccelPlan& p, int64_t ni, const void* xi, int64_t nj, const void* xj,
                        const void* mj, double eps, double G, int prec, void* acc, void* pot,
                        void* ws, size_t ws_bytes, hipStream_t s) {
    return timed(NB_PROF_FORCE, s, [&] {
        if (p.sym.waves)
            return launch_force_sym(prec, p.sym, ni, xi, mj, eps, G, acc, ws, ws_bytes, s,
                                    nullptr, 0.0, pot);
        return launch_force(prec, p.sh, ni, xi, nj, xj, mj, eps, G, p.self_set, acc, pot, ws, s);
    });
}

}  // namespace nb

namespace {

int accel_common(int64_t ni, const void* xi, int64_t nj, const void* xj, const void* mj,
                 double eps, double G, int prec, void* acc, void* pot, const nb_launch* launch,
                 void* ws, size_t ws_bytes, void* stream) {
    AccelPlan plan;
    int st = accel_plan(ni, xi, nj, xj, mj, eps, G, prec, acc, pot, launch, &plan);
    if (st != NB_OK) return st;
    if ((st = check_ws(ws, ws_bytes, plan.need)) != NB_OK) return st;
    // the bytes the pass may use: a banded pass uses what it is given, up to
    // every partial at once
    const size_t used = std::min(ws_bytes, plan.full);
    if (accel_ws_overlaps(ws, used, ni, xi, nj, xj, mj, prec, acc, pot)) return NB_EINVAL;
    if ((st = check_device()) != NB_OK) return st;
    return hip_status(accel_launch(plan, ni, xi, nj, xj, mj, eps, G, prec, acc, pot, ws, used,
                                   static_cast<hipStream_t>(stream)));
}

}  // namespace

extern "C" {

int nbody_accel(int64_t ni, const void* xi, int64_t nj, const void* xj, const void* mj, double eps,
                double G, int prec, void* acc, void* pot, void* ws, size_t ws_bytes, void* stream) {
    return accel_common(ni, xi, nj, xj, mj, eps, G, prec, acc, pot, nullptr, ws, ws_bytes, stream);
}

int nbody_accel_ex(int64_t ni, const void* xi, int64_t nj, const void* xj, const void* mj,
                   double eps, double G, int prec, void* acc, void* pot, const nb_launch* launch,
                   void* ws, size_t ws_bytes, void* stream) {
    return accel_common(ni, xi, nj, xj, mj, eps, G, prec, acc, pot, launch, ws, ws_bytes, stream);
}

int nbody_step(int64_t n, void* x, void* v, const void* m, void* acc, double eps, double G,
               double dt, int64_t nsteps, int prec, unsigned flags, void* ckpt, int64_t ckpt_every,
               void* ws, size_t ws_bytes, void* stream) {
    if (!valid_prec(prec)) return NB_EUNSUPPORTED;
    if (n < 1 || n > kMaxN || nsteps < 0) return NB_EINVAL;
    if (!valid_eps(eps, prec) || !isfinite(G) || !isfinite(dt)) return NB_EINVAL;
    if (flags & ~(NB_ACC_VALID | NB_GRAPH)) return NB_EINVAL;
    const size_t ps = pos_size(prec), ms = mass_size(prec);
    if (!x || !v || !m || !acc) return NB_EINVAL;
    if (!aligned(x, ps) || !aligned(v, ps) || !aligned(m, ms) || !aligned(acc, ps)) return NB_EINVAL;
    const size_t vb = 3 * (size_t)n * ps;
    if (overlaps(x, vb, v, vb) || overlaps(x, vb, acc, vb) || overlaps(v, vb, acc, vb) ||
        overlaps(m, (size_t)n * ms, x, vb) || overlaps(m, (size_t)n * ms, v, vb) ||
        overlaps(m, (size_t)n * ms, acc, vb))
        return NB_EINVAL;
    if (ckpt) {
        if (ckpt_every < 1 || !aligned(ckpt, ps)) return NB_EINVAL;
        const size_t cb = (size_t)(nsteps / ckpt_every + 1) * 3 * vb;
        if (overlaps(ckpt, cb, x, vb) || overlaps(ckpt, cb, v, vb) || overlaps(ckpt, cb, acc, vb))
            return NB_EINVAL;
    }
    const Shape sh = choose_force_shape(prec, n, n);
    const SymShape sym = choose_sym_shape(prec, n);
    const SymLayout L = sym.waves ? sym_layout(prec, sym, n) : SymLayout{};
    const size_t need = sym.waves ? sym_min_bytes(L) : accel_ws(sh, n);
    int st = check_ws(ws, ws_bytes, need);
    if (st != NB_OK) return st;
    const size_t used = sym.waves ? std::min(ws_bytes, sym_full_bytes(L)) : need;
    if (used && (overlaps(ws, used, x, vb) || overlaps(ws, used, v, vb) ||
                 overlaps(ws, used, m, (size_t)n * ms) || overlaps(ws, used, acc, vb) ||
                 (ckpt && overlaps(ws, used, ckpt, (size_t)(nsteps / ckpt_every + 1) * 3 * vb))))
        return NB_EINVAL;
    if ((st = check_device()) != NB_OK) return st;

    hipStream_t s = static_cast<hipStream_t>(stream);
    const double h = 0.5 * dt;
    // Enqueues the whole loop on q.
    auto enqueue = [&](hipStream_t q) -> hipError_t {
        // force(kick, drift): a <- a(x), and with kick the closing half-kick
        // v <- v + h a in the same launch group (the pair pass never reads
        // v); with drift also the next step's kick and drift, in the
        // finishing kernel, where the pass has one (*drifted tells)
        auto force = [&](bool kick, bool drift, bool* drifted) {
            return timed(NB_PROF_FORCE, q, [&] {
                void* kv = kick ? v : nullptr;
                void* dx = (kick && drift) ? x : nullptr;
                if (sym.waves)
                    return launch_force_sym(prec, sym, n, x, m, eps, G, acc, ws, used, q, kv, h, nullptr,
                                            dx, dt, drifted);
                return launch_force(prec, sh, n, x, n, x, m, eps, G, true, acc, nullptr, ws, q, kv,
                                    h, dx, dt, drifted);
            });
        };
        auto store = [&](int64_t slot) -> hipError_t {
            return timed(NB_PROF_COPY, q, [&] {
                char* base = static_cast<char*>(ckpt) + (size_t)slot * 3 * vb;
                hipError_t e = copy_state(base, x, vb, q);
                if (e == hipSuccess) e = copy_state(base + vb, v, vb, q);
                if (e == hipSuccess) e = copy_state(base + 2 * vb, acc, vb, q);
                return e;
            });
        };
        hipError_t e = hipSuccess;
        if (!(flags & NB_ACC_VALID)) e = force(false, false, nullptr);
        if (e == hipSuccess && ckpt) e = store(0);
        // a step's kick and drift run in the previous force pass's finishing
        // kernel unless that pass ended the call or a checkpoint slot, whose
        // stored state is the synchronised one
        bool drifted = false;
        for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
            if (!drifted)
                e = timed(NB_PROF_UPDATE, q, [&] { return launch_kick_drift(prec, n, x, v, acc, h, dt, q); });
            const bool stored = ckpt && (k + 1) % ckpt_every == 0;
            const bool fuse = (k + 1 < nsteps) && !stored;
            drifted = false;
            if (e == hipSuccess) e = force(true, fuse, &drifted);
            if (e == hipSuccess && stored) e = store((k + 1) / ckpt_every);
        }
        return e;
    };
    // NB_GRAPH: replay a cached graph of the loop, unless a profile is being
    // taken (it times each launch group) or s is itself being captured (the
    // launches then go into the caller's graph)
    if ((flags & NB_GRAPH) && !g_prof) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(s, &cap);
        if (e != hipSuccess) return hip_status(e);
        if (cap == hipStreamCaptureStatusNone) {
            StepKey key;
            memset(&key, 0, sizeof(key));
            if ((e = hipGetDevice(&key.dev)) != hipSuccess) return hip_status(e);
            key.prec = prec;
            key.flags = flags;
            key.n = n;
            key.nsteps = nsteps;
            key.ckpt_every = ckpt ? ckpt_every : 0;
            key.x = x;
            key.v = v;
            key.m = m;
            key.acc = acc;
            key.ckpt = ckpt;
            key.ws = ws;
            key.ws_bytes = ws_bytes;
            key.eps = eps;
            key.G = G;
            key.dt = dt;
            return hip_status(graph_launch(key, s, enqueue));
        }
    }
    return hip_status(enqueue(s));
}

int nbody_graph_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    hipError_t err = hipSuccess;
    for (GraphEntry& g : g_graphs) {
        hipError_t e = release_graph(g);
        if (err == hipSuccess) err = e;
    }
    g_graphs.clear();
    return hip_status(err);
}

}  // extern "C"

namespace {

int adjoint_common(int64_t n, void* x, void* v, const void* m, void* acc, void* lam_x,
                   void* lam_v, void* lam_m, double eps, double G, double dt, int64_t nsteps,
                   int prec, unsigned flags, const void* ckpt, int64_t ckpt_every,
                   int64_t step_end, const nb_launch* launch, void* ws, size_t ws_bytes,
                   void* stream) {
    if (!valid_prec(prec)) return NB_EUNSUPPORTED;
    if (n < 1 || n > kMaxN || nsteps < 0) return NB_EINVAL;
    if (!valid_eps(eps, prec) || !isfinite(G) || !isfinite(dt)) return NB_EINVAL;
    if (flags & ~(NB_ADJ_ENTRY_HALF | NB_ADJ_EXIT_FULL)) return NB_EINVAL;
    const size_t ps = pos_size(prec), ms = mass_size(prec);
    if (!x || !v || !m || !acc || !lam_x || !lam_v || !lam_m) return NB_EINVAL;
    if (!aligned(x, ps) || !aligned(v, ps) || !aligned(m, ms) || !aligned(acc, ps) ||
        !aligned(lam_x, ps) || !aligned(lam_v, ps) || !aligned(lam_m, 8))
        return NB_EINVAL;
    const size_t vb = 3 * (size_t)n * ps;
    const void* bufs[6] = {x, v, acc, lam_x, lam_v, lam_m};
    const size_t sizes[6] = {vb, vb, vb, vb, vb, (size_t)n * 8};
    for (int p = 0; p < 6; ++p) {
        if (overlaps(bufs[p], sizes[p], m, (size_t)n * ms)) return NB_EINVAL;
        for (int q = p + 1; q < 6; ++q)
            if (overlaps(bufs[p], sizes[p], bufs[q], sizes[q])) return NB_EINVAL;
    }
    if (ckpt) {
        if (ckpt_every < 1 || !aligned(ckpt, ps) || step_end < nsteps || step_end > kMaxN)
            return NB_EINVAL;
        const size_t cb = (size_t)(step_end / ckpt_every + 1) * 3 * vb;
        for (int p = 0; p < 6; ++p)
            if (overlaps(ckpt, cb, bufs[p], sizes[p])) return NB_EINVAL;
    }
    Shape sh;
    SymShape sym;
    int st = resolve_adjoint(prec, n, launch, &sym, &sh);
    if (st != NB_OK) return st;
    const size_t need = adjoint_partials_need(prec, sym, sh, n, true);
    st = check_ws(ws, ws_bytes, need);
    if (st != NB_OK) return st;
    const size_t used = sym.waves ? std::min(ws_bytes, sym_full_bytes(adjoint_sym_layout(prec, sym, n, true)))
                                  : need;
    if (used) {
        if (overlaps(ws, used, m, (size_t)n * ms)) return NB_EINVAL;
        for (int p = 0; p < 6; ++p)
            if (overlaps(ws, used, bufs[p], sizes[p])) return NB_EINVAL;
        if (ckpt && overlaps(ws, used, ckpt, (size_t)(step_end / ckpt_every + 1) * 3 * vb))
            return NB_EINVAL;
    }
    if ((st = check_device()) != NB_OK) return st;

    hipStream_t s = static_cast<hipStream_t>(stream);
    const double h = 0.5 * dt;
    double* lm = static_cast<double*>(lam_m);
    hipError_t e = hipSuccess;
    // fused(c, update_state, drift): one adjoint pass; with drift its
    // finishing kernel (where the pass has one) also applies the next step's
    // reverse drift, and `drifted` records that it did
    bool drifted = false;
    auto fused = [&](double c, bool update_state, bool drift) {
        drifted = false;
        return timed(NB_PROF_ADJOINT, s, [&] {
            void* dx = drift ? x : nullptr;
            if (sym.waves)
                return launch_adjoint_sym(prec, sym, n, x, m, lam_v, eps, G, c, update_state, h, acc, v,
                                          lam_x, lm, ws, used, s, dx, dt, &drifted);
            return launch_adjoint(prec, sh, n, x, m, lam_v, eps, G, c, update_state, h, acc, v, lam_x,
                                  lm, ws, s, dx, dt, &drifted);
        });
    };
    // the state walked back to at loop index k, and whether it is reloaded
    auto anchor_at = [&](int64_t k) {
        return k < nsteps && ckpt && ((step_end - 1 - k) % ckpt_every == 0);
    };
    if (flags & NB_ADJ_ENTRY_HALF) e = fused(h, false, nsteps > 0 && !anchor_at(0));
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        const int64_t step = step_end - 1 - k;  // absolute index of the state walked back to
        const bool anchor = anchor_at(k);
        const bool walked = drifted;  // the previous pass already did this step's reverse drift
        drifted = false;
        if (anchor) {
            e = timed(NB_PROF_UPDATE, s, [&] { return launch_axpy_pos(prec, 3 * n, lam_v, lam_x, dt, s); });
            const char* base = static_cast<const char*>(ckpt) + (size_t)(step / ckpt_every) * 3 * vb;
            if (e == hipSuccess)
                e = timed(NB_PROF_COPY, s, [&] {
                    hipError_t r = copy_state(x, base, vb, s);
                    if (r == hipSuccess) r = copy_state(v, base + vb, vb, s);
                    if (r == hipSuccess) r = copy_state(acc, base + 2 * vb, vb, s);
                    return r;
                });
        } else if (!walked) {
            e = timed(NB_PROF_UPDATE, s, [&] {
                return launch_reverse_drift(prec, n, x, v, acc, lam_x, lam_v, h, dt, s);
            });
        }
        const bool last = (k == nsteps - 1);
        const double c = last ? ((flags & NB_ADJ_EXIT_FULL) ? dt : h) : dt;
        if (e == hipSuccess) e = fused(c, !anchor, !last && !anchor_at(k + 1));
    }
    return hip_status(e);
}

}  // namespace

extern "C" {

int nbody_step_adjoint(int64_t n, void* x, void* v, const void* m, void* acc, void* lam_x,
                       void* lam_v, void* lam_m, double eps, double G, double dt, int64_t nsteps,
                       int prec, unsigned flags, const void* ckpt, int64_t ckpt_every,
                       int64_t step_end, void* ws, size_t ws_bytes, void* stream) {
    return adjoint_common(n, x, v, m, acc, lam_x, lam_v, lam_m, eps, G, dt, nsteps, prec, flags,
                          ckpt, ckpt_every, step_end, nullptr, ws, ws_bytes, stream);
}

int nbody_step_adjoint_ex(int64_t n, void* x, void* v, const void* m, void* acc, void* lam_x,
                          void* lam_v, void* lam_m, double eps, double G, double dt,
                          int64_t nsteps, int prec, unsigned flags, const void* ckpt,
                          int64_t ckpt_every, int64_t step_end, const nb_launch* launch,
                          void* ws, size_t ws_bytes, void* stream) {
    return adjoint_common(n, x, v, m, acc, lam_x, lam_v, lam_m, eps, G, dt, nsteps, prec, flags,
                          ckpt, ckpt_every, step_end, launch, ws, ws_bytes, stream);
}

int nbody_diag(int64_t n, const void* x, const void* v, const void* m, double eps, double G,
               int prec, double* out, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_prec(prec)) return NB_EUNSUPPORTED;
    if (n < 1 || n > kMaxN) return NB_EINVAL;
    if (!valid_eps(eps, prec) || !isfinite(G)) return NB_EINVAL;
    const size_t ps = pos_size(prec), ms = mass_size(prec);
    if (!x || !v || !m || !out) return NB_EINVAL;
    if (!aligned(x, ps) || !aligned(v, ps) || !aligned(m, ms) || !aligned(out, 8)) return NB_EINVAL;
    const size_t need = diag_workspace_bytes(n);
    int st = check_ws(ws, ws_bytes, need);
    if (st != NB_OK) return st;
    if (need && (overlaps(ws, need, x, 3 * (size_t)n * ps) || overlaps(ws, need, v, 3 * (size_t)n * ps) ||
                 overlaps(ws, need, m, (size_t)n * ms) || overlaps(ws, need, out, 13 * sizeof(double))))
        return NB_EINVAL;
    if ((st = check_device()) != NB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return hip_status(timed(NB_PROF_DIAG, s, [&] { return launch_diag(prec, n, x, v, m, eps, G, out, ws, s); }));
}

int diffusion3d_step(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                     double dt, double kappa, const float* f, float* fn, void* stream) {
    if (nx < 1 || ny < 1 || nz < 1 || nx > (int64_t(1) << 21) || ny > 524280) return NB_EINVAL;
    if (nx * ny > (int64_t(1) << 31) || nx * ny * nz > (int64_t(1) << 31) - 1) return NB_EINVAL;
    for (double h : {dx, dy, dz})
        if (!isfinite(h) || !(h > 0.0)) return NB_EINVAL;
    if (!isfinite(dt) || !isfinite(kappa)) return NB_EINVAL;
    if (!f || !fn || !aligned(f, 4) || !aligned(fn, 4)) return NB_EINVAL;
    const size_t bytes = (size_t)(nx * ny * nz) * sizeof(float);
    if (overlaps(f, bytes, fn, bytes)) return NB_EINVAL;
    int st = check_device();
    if (st != NB_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return hip_status(timed(NB_PROF_UPDATE, s, [&] {
        return launch_diffusion3d(nx, ny, nz, dx, dy, dz, dt, kappa, f, fn, s);
    }));
}

size_t nbody_pass_workspace_size(int op, int64_t ni, int64_t nj, int prec, int self_set,
                                 int potential, const nb_launch* launch) {
    if (!valid_prec(prec) || ni < 1 || nj < 1 || ni > kMaxN || nj > kMaxN) return 0;
    SymShape sym;
    Shape sh;
    if (op == NB_OP_ADJOINT) {
        if (ni != nj || resolve_adjoint(prec, ni, launch, &sym, &sh) != NB_OK) return 0;
        return adjoint_partials_need(prec, sym, sh, ni, false);
    }
    if (op != NB_OP_ACCEL || (self_set && ni != nj)) return 0;
    if (resolve_accel(prec, ni, nj, self_set != 0, potential != 0, launch, &sym, &sh) != NB_OK)
        return 0;
    if (sym.waves) return sym_default_bytes(sym_layout(prec, sym, ni, potential != 0));
    return accel_ws(sh, ni);
}

size_t nbody_workspace_size(int op, int64_t n, int prec) {
    if (!valid_prec(prec) || n < 1 || n > kMaxN) return 0;
    switch (op) {
    case NB_OP_ACCEL: {  // any ni, nj <= n; either pass, with or without the potential
        const size_t a = std::max(accel_ws(choose_force_shape(prec, n, n), n), force_partials_bound(n));
        const SymShape s0 = choose_sym_shape(prec, n), s1 = choose_sym_shape(prec, n, true);
        const size_t b = s0.waves ? sym_default_bytes(sym_layout(prec, s0, n)) : 0;
        const size_t c = s1.waves ? sym_default_bytes(sym_layout(prec, s1, n, true)) : 0;
        return std::max(a, std::max(b, c));
    }
    case NB_OP_STEP: {
        const SymShape sym = choose_sym_shape(prec, n);
        return sym.waves ? sym_default_bytes(sym_layout(prec, sym, n))
                         : accel_ws(choose_force_shape(prec, n, n), n);
    }
    case NB_OP_ADJOINT: {
        const SymShape sym = choose_adjoint_sym_shape(prec, n);
        if (sym.waves) return sym_default_bytes(adjoint_sym_layout(prec, sym, n, true));
        const Shape sh = choose_adjoint_shape(prec, n);
        return sh.split > 1 ? adjoint_partials_bytes(sh, n) : 0;
    }
    case NB_OP_DIAG:
        return diag_workspace_bytes(n);
    default:
        return 0;
    }
}

int nbody_pass_info(int op, int64_t n, int prec, nb_pass_info* out) {
    if (!out || n < 1 || n > kMaxN) return NB_EINVAL;
    if (!valid_prec(prec)) return NB_EUNSUPPORTED;
    nb_pass_info r;
    memset(&r, 0, sizeof(r));
    SymShape sym{0, 0};
    Shape sh{0, 0, 0};
    if (op == NB_OP_STEP) {
        sym = choose_sym_shape(prec, n);
        sh = choose_force_shape(prec, n, n);
    } else if (op == NB_OP_ADJOINT) {
        sym = choose_adjoint_sym_shape(prec, n);
        sh = choose_adjoint_shape(prec, n);
    } else {
        return NB_EINVAL;
    }
    if (sym.waves) {
        r.symmetric = 1;
        r.block = sym.waves * 64;
        r.i_per_lane = sym.ipl;
        r.split = 1;
        r.block_particles = (int64_t)sym.waves * 64 * sym.ipl;
    } else {
        r.block = sh.block;
        r.i_per_lane = sh.ipl;
        r.split = sh.split;
    }
    r.workspace_bytes = nbody_workspace_size(op, n, prec);
    *out = r;
    return NB_OK;
}

const char* nbody_strerror(int status) {
    switch (status) {
    case NB_OK: return "success";
    case NB_EINVAL: return "invalid argument";
    case NB_EWORKSPACE: return "workspace missing, misaligned or too small";
    case NB_EUNSUPPORTED: return "unsupported precision, operation or launch shape";
    case NB_ENODEV: return "no gfx950 device is current";
    case NB_EDEVICE: return "a HIP call failed";
    default: return "unknown status";
    }
}

int nbody_last_hip_error(void) { return g_last_hip_error; }

int nbody_profile_begin(void) {
    g_prof = true;
    return NB_OK;
}

int nbody_profile_end(nb_profile* out) {
    nb_profile p;
    memset(&p, 0, sizeof(p));
    hipError_t err = hipSuccess;
    for (const ProfRec& r : g_recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && err == hipSuccess) err = e;
        if (r.kind >= 0 && r.kind < NB_PROF_KINDS) {
            p.ms[r.kind] += ms;
            p.calls[r.kind] += 1;
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_prof = false;
    if (out) *out = p;
    return hip_status(err);
}

int nbody_device_info(char* buf, size_t len) {
    if (buf && len) buf[0] = 0;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return NB_ENODEV;
    }
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return NB_ENODEV;
    }
    if (buf && len)
        snprintf(buf, len, "%s %s, %d CUs, %d MHz, %.1f GiB, LDS %zu B/workgroup", p.name,
                 p.gcnArchName, p.multiProcessorCount, p.clockRate / 1000,
                 (double)p.totalGlobalMem / (1024.0 * 1024.0 * 1024.0), (size_t)p.sharedMemPerBlock);
    return strncmp(p.gcnArchName, "gfx950", 6) == 0 ? NB_OK : NB_ENODEV;
}

}  // extern "C"
