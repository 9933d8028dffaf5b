// The force-free passes of the symmetric adjoint (the entry pass of a
// reverse walk and every pass at a state reloaded from a checkpoint: J^T lam
// and G^T lam, no force sums), in a translation unit of their own so that
// they can be built with their own instruction schedule: the build compiles
// this file with the scheduler that groups memory clauses
// (-mllvm -amdgpu-sched-strategy=max-memory-clause). For the tile-
// compensated kernels it interleaves the sinks of a lane (159 VGPRs, three
// waves per SIMD, against
// 125 and four with the sinks one after another): 381.4 against 399.9 ms per
// pass at 2^20, 24.4 against 25.3 ms at 262144 (same boxes). The passes with
// the force sums lose under it (2^20: 507.6 against 491.7 ms), so they keep
// the default schedule. The plain FP32 policy's force-free passes gain too
// (262144: 23.8 against 25.1 ms); FP64's are the same either way (46.9
// against 46.8) and are built here with the others.
#include "adjoint_sym_pairs.h"

namespace nb {
namespace asym {

namespace {
template <class Pol>
hipError_t entry_any(const SymShape& sh, const ASymArgs<Pol>& a, hipStream_t stream) {
#define NB_ASYM_CASE(WV, KV) \
    if (sh.waves == WV && sh.ipl == KV) return launch_pairs<Pol, WV, KV, false>(a, stream);
    NB_ASYM_CASE(2, 2) NB_ASYM_CASE(4, 2) NB_ASYM_CASE(8, 2)
    NB_ASYM_CASE(4, 1) NB_ASYM_CASE(8, 1) NB_ASYM_CASE(2, 4) NB_ASYM_CASE(4, 4)
    NB_ASYM_CASE(8, 4)
    if constexpr (!std::is_same<typename Pol::calc_t, double>::value) {
        NB_ASYM_CASE(16, 2)  // FP64 in 16 waves would spill
    }
#undef NB_ASYM_CASE
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs<PolMixTileC>& a,
                              hipStream_t stream) {
    return entry_any(sh, a, stream);
}
hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs<PolF32>& a, hipStream_t stream) {
    return entry_any(sh, a, stream);
}
hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs<PolF64>& a, hipStream_t stream) {
    return entry_any(sh, a, stream);
}

}  // namespace asym
}  // namespace nb
