/*
 * diffusion3d.h -- C ABI of the 3-D diffusion step in libnbody.so (gfx950).
 *
 * The paper's second, memory-bound demonstration (section "3D diffusion
 * equation"): one explicit step of du/dt = kappa lap(u) on an
 * nx x ny x nz grid,
 *   fn = cc f + ce f(i+1) + cw f(i-1) + cn f(j+1) + cs f(j-1) + ct f(k+1) + cb f(k-1),
 *   ce = cw = kappa dt / dx^2, cn = cs = kappa dt / dy^2, ct = cb = kappa dt / dz^2,
 *   cc = 1 - (ce + cw + cn + cs + ct + cb),
 * where a neighbour outside the grid is replaced by the nearest point inside
 * (zero-flux boundary). The coefficients are formed in FP64 and rounded once
 * to FP32; the update is FP32.
 *
 * Layout: f and fn are FP32 device arrays of nx*ny*nz elements, point
 * (i, j, k) at index k + nz * (j + ny * i) (k fastest), 4-byte aligned,
 * caller-owned, not overlapping. The call only enqueues work on `stream`
 * (a hipStream_t, NULL = default stream) and returns.
 *
 * Returns NB_OK, or (nbody.h) NB_EINVAL for a size < 1, nx > 2^21,
 * ny > 524280, nx*ny*nz > 2^31 - 1, a non-finite or non-positive dx, dy, dz,
 * a non-finite dt or kappa, NULL, misaligned or overlapping arrays;
 * NB_ENODEV without a gfx950 device; NB_EDEVICE if the launch fails.
 * Arguments are checked before any HIP call.
 */
#ifndef DIFFUSION3D_H
#define DIFFUSION3D_H

#include <stdint.h>

#include "nbody.h"

#ifdef __cplusplus
extern "C" {
#endif

int diffusion3d_step(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                     double dt, double kappa, const float *f, float *fn, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DIFFUSION3D_H */
