/* Drives the FP64 oracle through every boundary type, viscosity law, normal scheme and
 * phase-field lattice on small grids, for a build with the address and undefined-behaviour
 * sanitizers (run by tests/test_oracle_sanitizers.py on the CPU). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny, bc_ylo, bc_yhi, visc_law, grad_scheme;
    double rho_l, rho_g, nu_l, nu_g, sigma, W, M, Gx, Gy;
    int32_t f_lattice, reserved;
} orc_params;
typedef struct orc_sim orc_sim;
orc_sim* orc_create(const orc_params* p, const double* phi0, const double* ux0, const double* uy0);
void orc_step(orc_sim* s, int64_t n);
void orc_moments(orc_sim* s, double* phi, double* rho, double* p, double* ux, double* uy);
void orc_destroy(orc_sim* s);

int main(void) {
    const int bcs[4][2] = {{0, 0}, {1, 1}, {1, 2}, {2, 1}};
    int runs = 0;
    for (int b = 0; b < 4; ++b)
        for (int law = 0; law < 3; ++law)
            for (int gs = 0; gs < 2; ++gs)
                for (int q = 0; q < 2; ++q) {
                    orc_params p = {13, 7, bcs[b][0], bcs[b][1], law, gs,
                                    1000.0, 1.0, 0.1, 0.3, 0.01, 4.0, 0.1, 1e-6, 0.0,
                                    q ? 5 : 9, 0};
                    const int n = p.nx * p.ny;
                    double* a = (double*)malloc(5 * n * sizeof(double));
                    for (int k = 0; k < n; ++k) {
                        a[k] = 0.2 + 0.6 * (double)((k * 37) % 11) / 10.0;
                        a[n + k] = 1e-3 * ((k % 5) - 2);
                        a[2 * n + k] = 1e-3 * ((k % 3) - 1);
                    }
                    orc_sim* s = orc_create(&p, a, a + n, a + 2 * n);
                    if (!s) return 2;
                    orc_step(s, 5);
                    orc_moments(s, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n);
                    orc_destroy(s);
                    free(a);
                    ++runs;
                }
    printf("sanitized oracle runs: %d\n", runs);
    return 0;
}
