/* A plain C consumer of the library's C ABI: compiled with -std=c99
 * -pedantic -Werror against include/ and linked against libnbody.so, it
 * calls the host-only entry points and the argument validation (which runs
 * before any device call), so it runs without a GPU. Prints "ok" and exits
 * 0 when every check holds. */
#include <stdio.h>
#include <string.h>

#include "diffusion3d.h"
#include "nbody.h"

static int failures = 0;

static void check(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

int main(void)
{
    nb_pass_info info;
    char buf[256];
    double out[16];
    check(strcmp(nbody_strerror(NB_OK), "success") == 0, "strerror(NB_OK)");
    check(nbody_workspace_size(NB_OP_ACCEL, 64, NB_F64) == 0, "one tile needs no workspace");
    check(nbody_workspace_size(NB_OP_DIAG, 1000, NB_F64) > 0, "diagnostics workspace");
    /* 2^20 on itself: FP64 running sums, then bands of 4 GiB of partials */
    check(nbody_workspace_size(NB_OP_STEP, 1 << 20, NB_MIX_TILEC) ==
              (size_t)3 * (1 << 20) * 8 + ((size_t)4 << 30),
          "symmetric step workspace at 2^20");
    memset(&info, 0, sizeof(info));
    check(nbody_pass_info(NB_OP_STEP, 1 << 20, NB_MIX_TILEC, &info) == NB_OK, "pass_info");
    check(info.symmetric == 1 && info.block_particles == 2048, "symmetric pass at 2^20");
    check(nbody_pass_info(NB_OP_STEP, 1000, NB_MIX_TILEC, &info) == NB_OK && info.symmetric == 0,
          "one-sided pass at 1000");
    check(nbody_pass_info(NB_OP_STEP, 0, NB_F64, &info) == NB_EINVAL, "pass_info n = 0");
    /* validation before any device call */
    check(nbody_accel(0, 0, 0, 0, 0, 0.1, 1.0, NB_F64, 0, 0, 0, 0, 0) == NB_EINVAL,
          "accel with n = 0");
    check(nbody_accel(8, 0, 8, 0, 0, 0.1, 1.0, 17, 0, 0, 0, 0, 0) == NB_EUNSUPPORTED,
          "accel with an unknown policy");
    check(nbody_step(8, 0, 0, 0, 0, 0.1, 1.0, 0.01, 1, NB_F64, 0, 0, 0, 0, 0, 0) == NB_EINVAL,
          "step with NULL state");
    check(nbody_diag(8, 0, 0, 0, 0.1, 1.0, NB_F64, out, 0, 0, 0) == NB_EINVAL, "diag with NULL state");
    check(diffusion3d_step(0, 4, 4, 1.0, 1.0, 1.0, 0.1, 1.0, 0, 0, 0) == NB_EINVAL,
          "diffusion with nx = 0");
    {
        const int st = nbody_device_info(buf, sizeof(buf));
        check(st == NB_OK || st == NB_ENODEV, "device_info");
    }
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
