/* A plain C program that drives the library on the GPU with no Python and
 * no torch: HIP runtime calls for device memory, then nbody_accel,
 * nbody_step (with NB_GRAPH) and nbody_diag through the C ABI.
 *
 *   abi_gpu_consumer IN OUT
 *   IN:  int64 n, int64 nsteps, double eps, double dt, then x[3n], v[3n]
 *        (double) and m[n] (float): the NB_MIX_TILEC layout
 *   OUT: a(x)[3n], then x[3n], v[3n], acc[3n] after nsteps leapfrog steps,
 *        then the 13 diagnostics of the final state (all double)
 * Exit status 0 on success; a message on stderr otherwise. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "nbody.h"

#define HIP_OK(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
            return 2;                                                         \
        }                                                                     \
    } while (0)

#define NB_OK_(call)                                                          \
    do {                                                                      \
        int s_ = (call);                                                      \
        if (s_ != NB_OK) {                                                    \
            fprintf(stderr, "%s: %s\n", #call, nbody_strerror(s_));           \
            return 3;                                                         \
        }                                                                     \
    } while (0)

static void *dev_alloc(size_t bytes)
{
    void *p = NULL;
    if (bytes && hipMalloc(&p, bytes) != hipSuccess) return NULL;
    return p;
}

int main(int argc, char **argv)
{
    int64_t n, nsteps;
    double eps, dt, diag[13];
    FILE *f;
    if (argc != 3) {
        fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
        return 1;
    }
    f = fopen(argv[1], "rb");
    if (!f || fread(&n, 8, 1, f) != 1 || fread(&nsteps, 8, 1, f) != 1 ||
        fread(&eps, 8, 1, f) != 1 || fread(&dt, 8, 1, f) != 1 || n < 1 || n > (1 << 24)) {
        fprintf(stderr, "bad input header\n");
        return 1;
    }
    {
        const size_t vb = 3 * (size_t)n * sizeof(double), mb = (size_t)n * sizeof(float);
        double *hx = malloc(vb), *hv = malloc(vb), *ha = malloc(vb);
        float *hm = malloc(mb);
        void *x, *v, *m, *a, *ws, *dd;
        size_t wsb;
        if (!hx || !hv || !ha || !hm) return 1;
        if (fread(hx, 1, vb, f) != vb || fread(hv, 1, vb, f) != vb || fread(hm, 1, mb, f) != mb) {
            fprintf(stderr, "short input\n");
            return 1;
        }
        fclose(f);
        wsb = nbody_workspace_size(NB_OP_ACCEL, n, NB_MIX_TILEC);
        if (nbody_workspace_size(NB_OP_STEP, n, NB_MIX_TILEC) > wsb)
            wsb = nbody_workspace_size(NB_OP_STEP, n, NB_MIX_TILEC);
        if (nbody_workspace_size(NB_OP_DIAG, n, NB_MIX_TILEC) > wsb)
            wsb = nbody_workspace_size(NB_OP_DIAG, n, NB_MIX_TILEC);
        x = dev_alloc(vb);
        v = dev_alloc(vb);
        a = dev_alloc(vb);
        m = dev_alloc(mb);
        ws = dev_alloc(wsb);
        dd = dev_alloc(13 * sizeof(double));
        if (!x || !v || !a || !m || (wsb && !ws) || !dd) {
            fprintf(stderr, "hipMalloc failed\n");
            return 2;
        }
        HIP_OK(hipMemcpy(x, hx, vb, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(v, hv, vb, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(m, hm, mb, hipMemcpyHostToDevice));
        NB_OK_(nbody_accel(n, x, n, x, m, eps, 1.0, NB_MIX_TILEC, a, NULL, ws, wsb, NULL));
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemcpy(ha, a, vb, hipMemcpyDeviceToHost));
        f = fopen(argv[2], "wb");
        if (!f || fwrite(ha, 1, vb, f) != vb) return 1;
        NB_OK_(nbody_step(n, x, v, m, a, eps, 1.0, dt, nsteps, NB_MIX_TILEC,
                          NB_ACC_VALID | NB_GRAPH, NULL, 0, ws, wsb, NULL));
        NB_OK_(nbody_diag(n, x, v, m, eps, 1.0, NB_MIX_TILEC, (double *)dd, ws, wsb, NULL));
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemcpy(diag, dd, sizeof(diag), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(hx, x, vb, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(hv, v, vb, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(ha, a, vb, hipMemcpyDeviceToHost));
        if (fwrite(hx, 1, vb, f) != vb || fwrite(hv, 1, vb, f) != vb || fwrite(ha, 1, vb, f) != vb ||
            fwrite(diag, 8, 13, f) != 13)
            return 1;
        fclose(f);
        NB_OK_(nbody_graph_cache_clear());
        HIP_OK(hipFree(x));
        HIP_OK(hipFree(v));
        HIP_OK(hipFree(a));
        HIP_OK(hipFree(m));
        if (ws) HIP_OK(hipFree(ws));
        HIP_OK(hipFree(dd));
        free(hx);
        free(hv);
        free(ha);
        free(hm);
    }
    return 0;
}
