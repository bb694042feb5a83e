/*
 * A plain C caller of libslh (no Python, no HIP headers): builds a 20x20
 * homogeneous box (sigma_s = 1, sigma_a = 0.1, unit source on the central
 * 2x2 cells, N_s = 1, 10^4 particles per pass, dt = 0.1, S_8), lets the
 * library allocate with hipMalloc on the default stream, advances three
 * steps, then prints the remap flux of every cell and the balance of the
 * last remap pass, one value per line with 17 significant digits.  With the
 * argument "steady" it solves the same box in steady state instead (one
 * step).  Exit status 0 on success; on error the library's message goes to
 * stderr.  Built by the package's build step; run by the GPU tests.
 */
#include <stdio.h>
#include <string.h>

#include "slh.h"

#define N 20

static int check(slh_status s, const char *what)
{
    if (s != SLH_OK) {
        fprintf(stderr, "%s failed (%d): %s\n", what, (int)s, slh_last_error());
        return 1;
    }
    return 0;
}

int main(int argc, char **argv)
{
    const int steady = argc > 1 && strcmp(argv[1], "steady") == 0;
    static double sig_s[N * N], sig_a[N * N], q[N * N], phi[N * N];
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            sig_s[j * N + i] = 1.0;
            sig_a[j * N + i] = 0.1;
            q[j * N + i] = (i >= 9 && i < 11 && j >= 9 && j < 11) ? 1.0 : 0.0;
        }
    slh_problem p;
    memset(&p, 0, sizeof p);
    p.abi_version = SLH_ABI_VERSION;
    p.nx = N;
    p.ny = N;
    p.x_lo = 0.0;
    p.x_hi = 2.0;
    p.y_lo = 0.0;
    p.y_hi = 2.0;
    p.sigma_s = sig_s;
    p.sigma_a = sig_a;
    p.q = q;
    p.c = 1.0;
    p.dt = 0.1;
    p.n_s = 1;
    p.n_particles = 10000;
    p.sn_order = 8;
    p.time_closure = 2.0;
    p.si_tol = 1e-12;
    p.si_max_iter = 400;
    p.w_cut_rel = 1e-8;
    p.seed = 20251116u;
    p.points = SLH_SOBOL_OWEN;
    p.precision = SLH_FP64;
    p.steady = steady;

    slh_solver *s = NULL;
    if (check(slh_create(&p, NULL, NULL, NULL, NULL, &s), "slh_create")) return 1;
    if (check(slh_advance(s, steady ? 1 : 3), "slh_advance")) return 1;
    if (check(slh_get_flux(s, SLH_FLUX_REMAP, phi), "slh_get_flux")) return 1;
    slh_balance b;
    if (check(slh_get_balance(s, 2, &b), "slh_get_balance")) return 1;
    for (int k = 0; k < N * N; ++k) printf("%.17g\n", phi[k]);
    printf("%.17g\n%.17g\n%llu\n", b.emitted, b.absorbed, (unsigned long long)b.segments);
    slh_destroy(s);
    return 0;
}
