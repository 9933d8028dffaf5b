// Host-side check of the band plan of the symmetric passes (csrc/common.h):
// for many layouts and workspace budgets, walks every band the library
// would launch, maps its work items to block pairs with the kernels' own
// band_item, replays every partial the pair kernel writes and every partial
// the fold kernel reads through the kernels' own SymBandView::offset, and
// checks that
//   * every block pair (I, J), I <= J, is one work item of exactly one band;
//   * a band's writes stay inside its partials, each element written once;
//   * every read finds the element written for that particle, quantity and
//     slot, in the same band;
//   * every particle receives its slots 0 .. nb-1 exactly once and in order;
//   * a band's partials fit the budget and it launches < 2^31 threads.
// No device is touched. Prints "ok" and exits 0, or names the failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "common.h"

using namespace nb;

static int fail(const char* what, long long a, long long b) {
    std::printf("FAIL: %s (%lld, %lld)\n", what, a, b);
    std::exit(1);
}

static void check(int64_t n, int64_t bi, int nq, size_t elem, size_t fin, size_t ws, int nt) {
    const SymLayout L{n, bi, (int)((n + bi - 1) / bi), nq, elem, fin};
    const SymPlan plan = sym_plan(L, ws, nt);
    if (!plan.valid) fail("workspace below the minimum", (long long)ws, 0);
    const bool one = plan.one;
    const size_t budget = plan.budget;
    if (!one && plan.parts + budget > ws) fail("partials past the workspace", (long long)ws, 0);
    if (!one && plan.parts < (size_t)nq * n * fin) fail("partials over the running sums", 0, 0);
    std::vector<int> pair_seen((size_t)L.nb * L.nb, 0);
    std::vector<int> next_slot((size_t)n, 0);  // next slot each particle must receive
    for (int I0 = 0; I0 < L.nb;) {
        const int I1 = sym_band_end(L, I0, budget, nt);
        if (I1 <= I0 || I1 > L.nb) fail("band end", I0, I1);
        if (one && !(I0 == 0 && I1 == L.nb)) fail("one band expected", I0, I1);
        const size_t bytes = sym_band_bytes(L, I0, I1);
        if (bytes > budget) fail("band over budget", (long long)bytes, (long long)budget);
        const int64_t items = sym_band_items(L, I0, I1);
        if (items * nt >= (int64_t(1) << 31)) fail("too many threads", items, nt);
        const SymBandView b = sym_band_view(L, I0, I1);
        const size_t elems = bytes / elem;
        // tag of the partial each element holds: (particle, quantity, slot)
        std::vector<long long> tag(elems, -1);
        auto put = [&](int k, int c, int p) {
            const size_t o = b.offset(k, c, p);
            if (o >= elems) fail("write outside the band", (long long)o, (long long)elems);
            if (tag[o] != -1) fail("element written twice", (long long)o, k);
            tag[o] = ((long long)p * nq + c) * L.nb + k;
        };
        for (int64_t t = 0; t < items; ++t) {
            int I, J;
            band_item(t, I0, I1, I, J);
            if (I < I0 || I >= I1 || J < I || J >= L.nb) fail("item outside the band", I, J);
            if (pair_seen[(size_t)I * L.nb + J]++) fail("block pair twice", I, J);
            for (int64_t p = I * bi; p < std::min(n, (I + 1) * bi); ++p)  // sink side: slot J
                for (int c = 0; c < nq; ++c) put(J, c, (int)p);
            if (I != J)
                for (int64_t p = J * bi; p < std::min(n, (J + 1) * bi); ++p)  // source side: slot I
                    for (int c = 0; c < nq; ++c) put(I, c, (int)p);
        }
        for (size_t o = 0; o < elems; ++o)
            if (tag[o] == -1) fail("element never written", (long long)o, I0);
        // the fold: particles base .. n-1, slots I0 .. I1-1, then the band's
        // own particles I1 .. nb-1
        for (int64_t p = b.base; p < n; ++p) {
            const bool own = p < b.base + b.nbp;
            for (int k = I0; k < (own ? L.nb : I1); ++k) {
                if (next_slot[p] != k) fail("slot out of order", p, k);
                for (int c = 0; c < nq; ++c)
                    if (tag[b.offset(k, c, (int)p)] != ((long long)p * nq + c) * L.nb + k)
                        fail("read a different partial", p, k);
                ++next_slot[p];
            }
        }
        I0 = I1;
    }
    for (int I = 0; I < L.nb; ++I)
        for (int J = I; J < L.nb; ++J)
            if (pair_seen[(size_t)I * L.nb + J] != 1) fail("block pair missed", I, J);
    for (int64_t p = 0; p < n; ++p)
        if (next_slot[p] != L.nb) fail("particle missed slots", p, next_slot[p]);
}

int main() {
    int cases = 0;
    for (int64_t n : {1, 63, 64, 65, 1000, 3001, 4096, 5000})
        for (int64_t bi : {64, 128, 256})
            for (int nq : {3, 4, 7})
                for (size_t elem : {4, 8}) {
                    const SymLayout L{n, bi, (int)((n + bi - 1) / bi), nq, elem, 8};
                    const size_t lo = sym_min_bytes(L), hi = sym_full_bytes(L);
                    for (int s = 0; s <= 6; ++s) {
                        const size_t ws = lo + (hi - lo) * s / 6;
                        check(n, bi, nq, elem, 8, ws, 256);
                        ++cases;
                    }
                    check(n, bi, nq, elem, 8, hi + 4096, 256);
                    // a thread limit that binds before the budget does (a
                    // workspace that holds every partial: the running sums
                    // then have to fit beside the bands)
                    check(n, bi, nq, elem, 8, hi + sym_run_bytes(L) + sym_band_bytes(L, 0, 1),
                          (int)((int64_t(1) << 31) / (L.nb + 2)));
                    cases += 2;
                }
    // the defaults the library asks for leave the budget above the minimum
    for (int64_t n : {int64_t(12288), int64_t(1) << 20, int64_t(3) << 20, int64_t(1) << 28})
        for (int nq : {3, 4, 7}) {
            const SymLayout L{n, 1024, (int)((n + 1023) / 1024), nq, 4, 8};
            if (sym_default_bytes(L) < sym_min_bytes(L)) fail("default below minimum", n, nq);
            if (sym_default_bytes(L) > sym_full_bytes(L) + sym_run_bytes(L)) fail("default too big", n, nq);
        }
    std::printf("ok %d\n", cases);
    return 0;
}
