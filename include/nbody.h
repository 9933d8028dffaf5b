/*
 * nbody.h -- C ABI of libnbody.so, a direct-summation gravitational N-body
 * library for AMD Instinct MI355X (gfx950).
 *
 * What it computes
 *   The softened pairwise acceleration of Eq. (1) of the paper (section
 *   "N-body simulation"),
 *       a_i = G * sum_j m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^(3/2),
 *   evaluated for a set of sinks i against a set of sources j (the paper's
 *   calc_acc takes Ni sinks and Nj sources), inside a second-order
 *   kick-drift-kick (KDK) leapfrog, with a reverse-mode adjoint of that
 *   leapfrog and FP64 energy / momentum diagnostics. The paper's listing
 *   includes the j = i term, which contributes exactly zero to a_i when
 *   eps > 0; so does this library.
 *
 * Data layout (all entry points)
 *   Structure of arrays. A position, velocity, acceleration or adjoint array
 *   of n particles is 3n contiguous elements: x[0..n), y[0..n), z[0..n).
 *   Masses and potentials are n elements. The element types are set by the
 *   precision policy `prec` (nb_prec below). Every pointer must be aligned to
 *   its element size. All device pointers are HIP device (or managed)
 *   memory owned by the caller; the library never allocates, frees or
 *   retains device memory for data (the HIP graphs that nbody_step keeps for
 *   NB_GRAPH are runtime objects, freed by nbody_graph_cache_clear()).
 *   Scratch memory comes from the caller's workspace `ws` (device memory,
 *   256-byte aligned, at least nbody_workspace_size() bytes; may be NULL
 *   when that size is 0). The part of the workspace a call uses must not
 *   overlap any other buffer of the call (NB_EINVAL).
 *
 * Pair passes and reproducibility
 *   The pair sums run in one of two forms, chosen by n and the policy
 *   (nbody_pass_info reports which): a one-sided kernel (every sink sums all
 *   sources; optional split of the source range with FP64 partials), or, for
 *   NB_MIX_TILEC, NB_F32 and NB_F64 with one set acting on itself from 12288
 *   particles (force and adjoint), a symmetric pass that evaluates each pair
 *   once for both bodies (Newton's third law) and adds partials per particle
 *   block (FP32; FP64 for NB_F64) in block order. No atomics in either: the
 *   same call on the same inputs gives bitwise the same results. Results of
 *   different forms or launch shapes differ by rounding only.
 *
 * Streams and synchronisation
 *   `stream` is a hipStream_t (NULL = the default stream). Every entry point
 *   only enqueues work on it and returns; nothing waits for the device. Two
 *   calls on different streams may run concurrently if they do not share
 *   writable buffers or workspace. Arguments are validated before any HIP
 *   call; a rejected call enqueues nothing.
 *
 * Errors
 *   Every entry point returns an nb_status. No C++ exception crosses the
 *   ABI. NB_EDEVICE means a HIP call failed; the HIP error is available via
 *   nbody_last_hip_error().
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nb_status {
    NB_OK = 0,
    NB_EINVAL = 1,       /* invalid argument (see each entry point)           */
    NB_EWORKSPACE = 2,   /* workspace NULL, misaligned or smaller than needed */
    NB_EUNSUPPORTED = 3, /* precision / operation / launch shape not provided */
    NB_ENODEV = 4,       /* no gfx950 device is current                        */
    NB_EDEVICE = 5       /* a HIP call failed (launch or copy)                 */
} nb_status;

/*
 * Precision policies. "pos" is the element type of positions, velocities,
 * accelerations, potentials and position/velocity adjoints; "mass" that of
 * masses; the mass adjoint is always double.
 *
 *   NB_F64        pos double, mass double. Pair arithmetic and sums in FP64
 *                 (hardware reciprocal square root refined to ~1 ulp by one
 *                 third-order step).
 *   NB_F32        pos float,  mass float.  Pair arithmetic in FP32 with the
 *                 hardware reciprocal square root; per-particle sums are FP32
 *                 running sums, as the paper's listing (in the symmetric
 *                 pass, for a set on itself from 12288 particles, FP32 sums
 *                 over each source block, then over the blocks in FP32).
 *   NB_MIX_ACC32  pos double, mass float. Pair arithmetic in FP32 (as
 *                 NB_F32) on positions taken relative to an origin o, the
 *                 FP64 centroid of the sinks one workgroup owns (a
 *                 contiguous index range), and then rounded: the rounding
 *                 error of a separation is at most 2^-24 (|x_i - o| +
 *                 |x_j - o|), independent of where the system sits. FP32
 *                 running sums. Kick, drift and everything O(N) stay in FP64.
 *   NB_MIX_KAHAN  as NB_MIX_ACC32, but each running sum is Kahan-compensated
 *                 in FP32.
 *   NB_MIX_ACC64  as NB_MIX_ACC32, but each FP32 pair term is summed in FP64.
 *   NB_MIX_TILEC  as NB_MIX_ACC32, but the FP32 running sum restarts at every
 *                 j-tile and the tile sums are added in FP64. In the
 *                 symmetric passes the tiles are the source blocks (up to
 *                 4096 particles): a particle's partial from one block is an
 *                 FP32 sum (the passes with up to four sinks per lane for
 *                 the force, two for the adjoint, fold the sink side into
 *                 FP64 every 64 sources), and a particle's partials are
 *                 added in FP64.
 */
typedef enum nb_prec {
    NB_F64 = 0,
    NB_F32 = 1,
    NB_MIX_ACC32 = 2,
    NB_MIX_KAHAN = 3,
    NB_MIX_ACC64 = 4,
    NB_MIX_TILEC = 5
} nb_prec;

/* Operation codes for nbody_workspace_size(). */
typedef enum nb_op {
    NB_OP_ACCEL = 0,
    NB_OP_STEP = 1,
    NB_OP_ADJOINT = 2,
    NB_OP_DIAG = 3
} nb_op;

/* nbody_step() flags */
#define NB_ACC_VALID 0x1u      /* acc already holds a(x) on entry            */
#define NB_GRAPH 0x2u          /* replay the loop as an instantiated HIP graph
                                  (see nbody_step)                            */

/* nbody_step_adjoint() flags */
#define NB_ADJ_ENTRY_HALF 0x1u /* apply the h-weighted position adjoint at the
                                  entry state (set on the call that starts a
                                  backward pass at the rollout's last step)   */
#define NB_ADJ_EXIT_FULL 0x2u  /* weight the position adjoint at the exit
                                  state by dt instead of h (set on every call
                                  that does not end at the rollout's step 0)  */

/* Explicit launch shape for nbody_accel_ex() and nbody_step_adjoint_ex();
 * 0 in a field = library choice.
 *   symmetric = 0: the one-sided kernel (every sink sums every source)
 *     i_per_lane  sinks per lane: 1, 2 or 4 (adjoint: 1 or 2)
 *     block       threads per workgroup (= j-tile length): 64, 128, 256, 512
 *                 or 1024 (adjoint: up to 512)
 *     split       j-split: number of source ranges per sink, 1..256; partial
 *                 sums are combined in a fixed order
 *   symmetric = 1: the symmetric (third-law) pass of one set on itself
 *                 (NB_MIX_TILEC, NB_F32, NB_F64)
 *     block       threads per workgroup, waves x 64; with i_per_lane sinks
 *                 per lane, blocks of block x i_per_lane particles. Shapes
 *                 (block, i_per_lane): force (128, 2), (256, 2), (512, 2),
 *                 (1024, 2), (128, 4), (256, 4), (512, 4), (1024, 4), (128, 8),
 *                 (256, 8), (512, 8);
 *                 adjoint (128, 2), (256, 2), (512, 2), (1024, 2) (not
 *                 NB_F64), (256, 1), (512, 1), (128, 4), (256, 4), (512, 4)
 *                 (with eight sinks per
 *                 lane for the force, and four for the adjoint, each sink's
 *                 sum in NB_MIX_TILEC is an FP32 running sum over the source
 *                 block, as the source side's always is)
 *     split       must be 0 or 1
 * Other shapes: NB_EUNSUPPORTED. */
typedef struct nb_launch {
    int32_t i_per_lane;
    int32_t block;
    int32_t split;
    int32_t symmetric;
} nb_launch;

/*
 * nbody_accel -- accelerations of ni sinks from nj sources, Eq. (1).
 *
 *   xi   [3*ni] pos   sink positions (device)
 *   xj   [3*nj] pos   source positions (device); xi == xj with ni == nj means
 *                     one set acting on itself
 *   mj   [nj]   mass  source masses (device)
 *   eps  softening length: finite and > 0 (>= 2^-40 in the FP32 policies)
 *   G    gravitational constant, finite
 *   acc  [3*ni] pos   output accelerations (device); must not overlap inputs
 *   pot  [ni]   pos   optional output (NULL to skip): the potential
 *                     phi_i = -G sum_j m_j / sqrt(|r_j - r_i|^2 + eps^2),
 *                     with the j = i term removed when xi == xj (the paper's
 *                     CALCULATE_POTENTIAL branch sums it in; here it is
 *                     subtracted once per sink after the sum). In the
 *                     symmetric pass the potential of a pair comes from the
 *                     same reciprocal square root as its forces
 *   ws, ws_bytes      workspace, nbody_workspace_size(NB_OP_ACCEL, max(ni,nj), prec)
 *   stream            hipStream_t
 * Returns NB_EINVAL for ni < 1, nj < 1, ni or nj > 2^30, bad eps or G, a
 * NULL or misaligned pointer, or xi == xj with ni != nj.
 */
int nbody_accel(int64_t ni, const void *xi, int64_t nj, const void *xj,
                const void *mj, double eps, double G, int prec, void *acc,
                void *pot, void *ws, size_t ws_bytes, void *stream);

/*
 * nbody_accel_noalloc -- nbody_accel for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): no workspace argument and no allocation by the library.
 * The pass, its kernels and its results are those of nbody_accel for the same
 * arguments (bitwise); its scratch is a device array of the library of
 * NB_NOALLOC_SCRATCH_BYTES (128 MiB), one per device, held from the library's
 * first use on that device until the process ends. Arguments and errors as
 * nbody_accel, plus NB_EWORKSPACE when the pass needs more scratch than that:
 * the symmetric pass of a set on itself runs in bands within the array (see
 * nbody_workspace_size) and needs the running sums and one block row, which
 * fit up to about 2.8 million particles with the tile-compensated policy (2.1
 * million with the potential), 3.7 million with FP32 and 1.9 million with
 * FP64; separate sets, and sets below 12288 particles, need 4 x 8 x split x
 * ni bytes for the library's source split (none for large ni). Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (on different streams, or from different threads) race on it and
 * must be ordered by the caller. Nothing in the array needs clearing
 * between calls.
 */
#define NB_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int nbody_accel_noalloc(int64_t ni, const void *xi, int64_t nj, const void *xj,
                        const void *mj, double eps, double G, int prec, void *acc,
                        void *pot, void *stream);

/*
 * nbody_accel_ex -- nbody_accel with an explicit launch shape (for tuning and
 * for tests that a result does not depend on the shape). NULL launch = the
 * library's choice. NB_EUNSUPPORTED for a shape outside nb_launch's limits,
 * or a symmetric shape for separate sets or a policy without that pass.
 */
int nbody_accel_ex(int64_t ni, const void *xi, int64_t nj, const void *xj,
                   const void *mj, double eps, double G, int prec, void *acc,
                   void *pot, const nb_launch *launch, void *ws,
                   size_t ws_bytes, void *stream);

/*
 * nbody_step -- nsteps KDK leapfrog steps of size dt (h = dt/2), in place:
 *   v <- v + h a(x);  x <- x + dt v;  a <- a(x);  v <- v + h a,
 * the pair forces of Eq. (1) with the j = i term (zero) included.
 *
 *   n          particle count, 1..2^30
 *   x, v [3n]  pos, in/out (device)
 *   m    [n]   mass (device)
 *   acc  [3n]  pos, in/out: on entry a(x) if flags has NB_ACC_VALID (else it
 *              is computed first); on exit a(x) of the final state
 *   eps, G     as nbody_accel;  dt finite;  nsteps >= 0
 *   ckpt       optional (NULL to skip) device buffer of
 *              (nsteps / ckpt_every + 1) slots of 9n pos elements; slot k
 *              receives x, v, acc (3n each, in that order) at step
 *              k * ckpt_every, slot 0 being the entry state
 *   ckpt_every checkpoint interval >= 1 (ignored when ckpt is NULL)
 *   ws         workspace of nbody_workspace_size(NB_OP_STEP, n, prec) bytes
 *   flags      NB_ACC_VALID, NB_GRAPH
 *
 * NB_GRAPH: the 2 nsteps (+1) launches of the loop are recorded once into a
 * HIP graph on a capture stream owned by the library, instantiated, and
 * launched on `stream`; a later call with the same arguments (device,
 * pointers, sizes, eps, G, dt, nsteps, prec, flags) launches the cached
 * graph again, which saves the per-launch host cost when n is small. The
 * results are bitwise those of the same call without NB_GRAPH. Up to 16
 * graphs are kept per process (least recently used evicted, after its last
 * launch has finished); instantiation allocates HIP runtime objects, held
 * until nbody_graph_cache_clear() or process end. The flag is ignored while
 * a profile is being taken (nbody_profile_begin) and when `stream` is itself
 * being captured (the launches then go into the caller's graph).
 */
int nbody_step(int64_t n, void *x, void *v, const void *m, void *acc,
               double eps, double G, double dt, int64_t nsteps, int prec,
               unsigned flags, void *ckpt, int64_t ckpt_every, void *ws,
               size_t ws_bytes, void *stream);

/*
 * nbody_graph_cache_clear -- waits for the last launch of every graph that
 * nbody_step cached for NB_GRAPH and frees them. NB_EDEVICE if a HIP call
 * failed (the cache is emptied either way).
 */
int nbody_graph_cache_clear(void);

/*
 * nbody_step_adjoint -- reverse-mode derivative of nbody_step, walking
 * nsteps steps back from the entry state.
 *
 * On entry (x, v, acc) is the forward state at step k = step_end and
 * (lam_x, lam_v) = dL/dx_k, dL/dv_k. On exit (x, v, acc) is the state at
 * step k - nsteps and (lam_x, lam_v) = dL/dx, dL/dv there; lam_m has the
 * mass derivative of those steps added. Per step n+1 -> n:
 *   lam_v += dt lam_x;
 *   the state is walked back by the time-reversed KDK step, or, when ckpt is
 *   given and n is a multiple of ckpt_every, reloaded from slot n/ckpt_every;
 *   lam_x += c J(x_n)^T lam_v and lam_m += c G(x_n)^T lam_v, where J and G
 *   are the Jacobians of a(x, m) with respect to positions and masses,
 *   c = dt inside the walk, and c = h or dt at the exit state
 *   (NB_ADJ_EXIT_FULL). With NB_ADJ_ENTRY_HALF the same update with c = h is
 *   first applied at the entry state.
 *
 *   lam_x, lam_v [3n] pos, in/out; lam_m [n] double, in/out (accumulates)
 *   ckpt, ckpt_every  as written by nbody_step over the same rollout, or NULL
 *   step_end   absolute step index of the entry state (used with ckpt only);
 *              0 <= step_end - nsteps
 *   other arguments as nbody_step; ws of nbody_workspace_size(NB_OP_ADJOINT)
 */
int nbody_step_adjoint(int64_t n, void *x, void *v, const void *m, void *acc,
                       void *lam_x, void *lam_v, void *lam_m, double eps,
                       double G, double dt, int64_t nsteps, int prec,
                       unsigned flags, const void *ckpt, int64_t ckpt_every,
                       int64_t step_end, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * nbody_step_adjoint_ex -- nbody_step_adjoint with an explicit launch shape
 * for its fused adjoint pair passes (tuning, shape-invariance tests); NULL
 * launch = the library's choice. NB_EUNSUPPORTED as nbody_accel_ex. The
 * workspace is that of the shape: nbody_pass_workspace_size(NB_OP_ADJOINT,
 * n, n, prec, 1, 0, launch).
 */
int nbody_step_adjoint_ex(int64_t n, void *x, void *v, const void *m, void *acc,
                          void *lam_x, void *lam_v, void *lam_m, double eps,
                          double G, double dt, int64_t nsteps, int prec,
                          unsigned flags, const void *ckpt, int64_t ckpt_every,
                          int64_t step_end, const nb_launch *launch, void *ws,
                          size_t ws_bytes, void *stream);

/*
 * nbody_diag -- FP64 conserved quantities of a state (any policy; FP32
 * inputs are promoted exactly). out (device, 13 doubles):
 *   0 KE = 1/2 sum m|v|^2       1 PE = -G sum_{i<j} m_i m_j / sqrt(s_ij)
 *   2 E = KE + PE               3..5 P = sum m v
 *   6..8 L = sum m r x v        9..11 centre of mass     12 total mass
 * ws of nbody_workspace_size(NB_OP_DIAG, n, prec) bytes.
 */
int nbody_diag(int64_t n, const void *x, const void *v, const void *m,
               double eps, double G, int prec, double *out, void *ws,
               size_t ws_bytes, void *stream);

/*
 * Device-time profile of the library's own launches (tooling; not part of the
 * method). Between nbody_profile_begin() and nbody_profile_end() the calling
 * thread's entry points record a HIP event before and after each group of
 * launches of one kind, on the stream they launch on. nbody_profile_end()
 * waits for those events, fills *out (may be NULL) and stops recording.
 * Kinds: the pair-force kernel (with its split reduction), the fused adjoint
 * kernel (with its split reduction), O(N) leapfrog updates, diagnostics,
 * checkpoint copies. Not for use under stream capture.
 */
enum { NB_PROF_FORCE = 0, NB_PROF_ADJOINT = 1, NB_PROF_UPDATE = 2, NB_PROF_DIAG = 3,
       NB_PROF_COPY = 4, NB_PROF_KINDS = 5 };
typedef struct nb_profile {
    double ms[NB_PROF_KINDS];       /* summed device milliseconds per kind    */
    int64_t calls[NB_PROF_KINDS];   /* timed launch groups per kind           */
} nb_profile;
int nbody_profile_begin(void);
int nbody_profile_end(nb_profile *out);

/* Workspace bytes an operation asks for, for n particles (0 = none). For
 * NB_OP_ACCEL pass max(ni, nj): the size covers every call whose ni and nj
 * are both <= n (a small sink set against many sources takes the most
 * source ranges: up to 512 MiB of partials from n = 2^19 on). Returns 0 for
 * an invalid op or prec.
 * The symmetric passes take less as well: with a workspace that holds every
 * partial of the pass at once they run as one launch group; with less, in
 * bands of block rows, each followed by a kernel that adds the band's
 * partials to running sums per particle (kept at the start of the
 * workspace) in the same order -- bitwise the same results, at the cost of
 * more launches. The size asked for holds every partial up to 4 GiB of them,
 * else the running sums and 4 GiB (or one block row, if more) per band; a
 * call rejects a workspace that cannot hold the running sums and one block
 * row (NB_EWORKSPACE), and uses no more than every partial at once. */
size_t nbody_workspace_size(int op, int64_t n, int prec);

/* The workspace bytes one call asks for. op NB_OP_ACCEL: nbody_accel
 * (launch == NULL) or nbody_accel_ex with ni sinks, nj sources, self_set
 * nonzero when xi == xj (then ni == nj), potential nonzero when pot is given.
 * op NB_OP_ADJOINT: nbody_step_adjoint(_ex) of ni == nj particles (self_set
 * and potential ignored). 0 when none is needed or the arguments are
 * invalid. */
size_t nbody_pass_workspace_size(int op, int64_t ni, int64_t nj, int prec, int self_set,
                                 int potential, const nb_launch *launch);

/*
 * nbody_pass_info -- the pair pass the library runs for n particles acting
 * on themselves (op NB_OP_STEP: the force of a leapfrog, and of
 * nbody_accel with xi == xj and no explicit shape -- with a potential the
 * same shape, with four partials per particle in the symmetric pass; op
 * NB_OP_ADJOINT: the fused adjoint pass of nbody_step_adjoint). Host-side
 * only (no device needed). NB_EINVAL for another op, n outside 1..2^30 or a
 * NULL out; NB_EUNSUPPORTED for an unknown prec.
 *
 * symmetric = 1: the third-law pass -- particles cut into blocks of
 * block_particles = block * i_per_lane, one workgroup per block pair,
 * partials per block (FP32; FP64 for NB_F64) added in a fixed order
 * (NB_MIX_TILEC, NB_F32 and NB_F64, from 12288 up to 2^28 particles; from
 * 2^18 the force takes blocks of 2048 particles and the adjoint blocks of
 * 1024 at every n; the partials are written and folded in bands of the
 * workspace).
 * symmetric = 0: the one-sided kernel in the shape (i_per_lane, block,
 * split).
 */
typedef struct nb_pass_info {
    int32_t symmetric;
    int32_t block;           /* threads per workgroup                        */
    int32_t i_per_lane;      /* sinks per lane                               */
    int32_t split;           /* source ranges per sink (one-sided kernel)    */
    int64_t block_particles; /* particles per block (symmetric), else 0      */
    size_t workspace_bytes;  /* = nbody_workspace_size(op, n, prec)          */
} nb_pass_info;
int nbody_pass_info(int op, int64_t n, int prec, nb_pass_info *out);

/* Static text for a status code. */
const char *nbody_strerror(int status);

/* The last HIP error code this thread saw inside the library (0 if none). */
int nbody_last_hip_error(void);

/* Writes a one-line description of the current device into buf (always
 * NUL-terminated when len > 0). NB_ENODEV when no gfx950 device is there. */
int nbody_device_info(char *buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
