/*
 * A plain C consumer of the library (no Python, no torch): one 32^3 problem with an air
 * bubble in water (density ratio 1000, surface tension), solved in mixed precision with
 * the bubble deflated, then checked on the host against the library's own right-hand
 * side and operator: ||b - A p|| / ||b|| with b from mpp_rhs and A p from
 * mpp_apply_stencil.  Prints one JSON line; exit status 0 when the checks pass.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "mpp.h"

static int hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        return 0;
    }
    return 1;
}

int main(void) {
    const int n = 32;
    const size_t cells = (size_t)n * n * n, bytes = cells * sizeof(double);
    double *phi = malloc(bytes), *f = malloc(bytes), *b = malloc(bytes), *ap = malloc(bytes),
           *p = malloc(bytes);
    if (!phi || !f || !b || !ap || !p) return 2;
    /* the bubble: phi > 0 inside (the "+" side, air), a signed distance */
    const double cx = 0.5, cy = 0.45, cz = 0.55, r = 0.22, h = 1.0 / n;
    uint64_t s = 12345u;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const size_t c = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * k);
                const double x = (i + 0.5) * h - cx, y = (j + 0.5) * h - cy, z = (k + 0.5) * h - cz;
                phi[c] = r - sqrt(x * x + y * y + z * z);
                s = s * 6364136223846793005ull + 1442695040888963407ull; /* a 64-bit LCG */
                f[c] = 2.0 * (double)(s >> 11) / 9007199254740992.0 - 1.0;
            }
    const double rho_neg = 1.0, rho_pos = 1e-3, sigma = 0.01;
    double *d_phi, *d_f, *d_p, *d_b, *d_ap;
    void *ws;
    mpp_desc desc = {n, 1, 0u};
    const size_t wsb = mpp_workspace_bytes(&desc);
    if (!wsb) return 2;
    if (!hip_ok(hipMalloc((void **)&d_phi, bytes), "hipMalloc") ||
        !hip_ok(hipMalloc((void **)&d_f, bytes), "hipMalloc") ||
        !hip_ok(hipMalloc((void **)&d_p, bytes), "hipMalloc") ||
        !hip_ok(hipMalloc((void **)&d_b, bytes), "hipMalloc") ||
        !hip_ok(hipMalloc((void **)&d_ap, bytes), "hipMalloc") ||
        !hip_ok(hipMalloc(&ws, wsb), "hipMalloc"))
        return 2;
    if (!hip_ok(hipMemcpy(d_phi, phi, bytes, hipMemcpyHostToDevice), "hipMemcpy") ||
        !hip_ok(hipMemcpy(d_f, f, bytes, hipMemcpyHostToDevice), "hipMemcpy"))
        return 2;
    mpp_op op = NULL;
    int st = mpp_build_operator(&desc, d_phi, &rho_neg, &rho_pos, &sigma, ws, wsb, NULL, &op);
    if (st != MPP_OK) {
        printf("{\"stage\": \"build\", \"status\": %d}\n", st);
        return 1;
    }
    mpp_solve_opts o;
    mpp_default_opts(&o);
    o.mode = MPP_MODE_MIXED;
    o.rtol = 1e-10;
    mpp_solve_info info;
    st = mpp_solve(op, d_f, d_p, &o, &info, NULL);
    int st2 = mpp_rhs(op, d_f, d_b, NULL, NULL);
    int st3 = mpp_apply_stencil(op, d_p, d_ap, NULL);
    if (!hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize") ||
        !hip_ok(hipMemcpy(b, d_b, bytes, hipMemcpyDeviceToHost), "hipMemcpy") ||
        !hip_ok(hipMemcpy(ap, d_ap, bytes, hipMemcpyDeviceToHost), "hipMemcpy") ||
        !hip_ok(hipMemcpy(p, d_p, bytes, hipMemcpyDeviceToHost), "hipMemcpy"))
        return 2;
    double rr = 0.0, bb = 0.0, mean = 0.0, pmax = 0.0;
    for (size_t c = 0; c < cells; ++c) {
        const double d = b[c] - ap[c];
        rr += d * d;
        bb += b[c] * b[c];
        mean += p[c];
        if (fabs(p[c]) > pmax) pmax = fabs(p[c]);
    }
    mean /= (double)cells;
    const double rel = sqrt(rr / bb);
    const int ok = st == MPP_OK && st2 == MPP_OK && st3 == MPP_OK && info.status == MPP_OK &&
                   rel <= 1.05e-10 && fabs(info.rel_resid - rel) <= 0.05 * rel + 1e-13 &&
                   fabs(mean) <= 1e-12 * pmax;
    printf("{\"status\": %d, \"iters\": %d, \"outer_iters\": %d, \"lib_rel_resid\": %.6e, "
           "\"host_rel_resid\": %.6e, \"mean_p\": %.3e, \"ok\": %d}\n",
           st, info.iters, info.outer_iters, info.rel_resid, rel, mean, ok);
    mpp_destroy_operator(op);
    hipFree(ws);
    hipFree(d_ap);
    hipFree(d_b);
    hipFree(d_p);
    hipFree(d_f);
    hipFree(d_phi);
    free(p);
    free(ap);
    free(b);
    free(f);
    free(phi);
    return ok ? 0 : 1;
}
