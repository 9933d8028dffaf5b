// The force-free passes of the symmetric adjoint (the entry pass of a reverse
// walk and every pass at a state reloaded from a checkpoint: J^T lam and
// G^T lam, no force sums), in a translation unit of their own so that they
// can be built with their own instruction schedule: the build compiles this
// file with the scheduler that groups memory clauses
// (-mllvm -amdgpu-sched-strategy=max-memory-clause). For these kernels it
// interleaves the sinks of a lane (159 VGPRs, three waves per SIMD, against
// 125 and four with the sinks one after another): 381.4 against 399.9 ms per
// pass at 2^20, 24.4 against 25.3 ms at 262144 (same boxes). The passes with
// the force sums lose under it (2^20: 507.6 against 491.7 ms), so they keep
// the default schedule.
#include "adjoint_sym_pairs.h"

namespace nb {
namespace asym {

hipError_t launch_pairs_entry(const SymShape& sh, const ASymArgs& a, hipStream_t stream) {
#define NB_ASYM_CASE(WV, KV) \
    if (sh.waves == WV && sh.ipl == KV) return launch_pairs<WV, KV, false>(a, stream);
    NB_ASYM_CASE(2, 2) NB_ASYM_CASE(4, 2) NB_ASYM_CASE(8, 2) NB_ASYM_CASE(16, 2)
    NB_ASYM_CASE(4, 1) NB_ASYM_CASE(8, 1) NB_ASYM_CASE(2, 4) NB_ASYM_CASE(4, 4)
    NB_ASYM_CASE(8, 4)
#undef NB_ASYM_CASE
    return hipErrorInvalidValue;
}

}  // namespace asym
}  // namespace nb
