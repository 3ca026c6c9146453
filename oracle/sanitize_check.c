/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A small driver that runs every entry point of the CPU oracle
 * (lbm_oracle.c) on small channels, for a build with the address and
 * undefined-behaviour sanitizers (tests/test_oracle_sanitizers.py compiles
 * it together with lbm_oracle.c, runs it and requires a clean exit with no
 * sanitizer report).  The channels cover the ghost rows at both walls, a
 * lattice only four cells high, unequal densities, viscosities and
 * conductivities, and a perturbed start, so that every stencil, wall link and
 * property path is taken.  Prints one line per case and the largest
 * magnitude seen (a finite number); exits non-zero on a failed call or a
 * non-finite value.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nx, ny, n_waves;
    double b, W, M_phi;
    double rho_a, rho_b, mu_a, mu_b, k_a, k_b;
    double sigma0, sigma_T, sigma_TT, T_ref;
    double T_h, dT, T_c;
    double Fx_ext, Fy_ext;
    double p0;
} params;

int orc_init_cold(const params* P, double* pop);
int orc_init_fields(const params* P, const double* phi, const double* ux, const double* uy, const double* T,
                    double* pop);
int orc_run(const params* P, double* pop, long nsteps);
int orc_macros(const params* P, const double* pop, double* phi, double* ux, double* uy, double* T, double* p);
void orc_build_F(double ux, double uy, double F[9][9]);
void orc_tables(double* P, double* Pinv, double* w, int* ex, int* ey);
void orc_collide_f_node(const double* f, double phi, double ux, double uy, double nxv, double nyv, double theta,
                        double M, double w_phi, double* out);
void orc_collide_g_node(const double* g, double p, double rho, double ux, double uy, double Ftx, double Fty,
                        double Fpx, double Fpy, double w_nu, double* out);
void orc_collide_h_node(const double* h, double T, double ux, double uy, double w_T, double* out);
void orc_set_threads(int n);

static params base(int nx, int ny, double b) {
    params p = {nx, ny, 1, b, 4.0, 0.02, 1.0, 1.0, 0.1, 0.1, 0.1, 0.1, 5e-3, -1e-4, 2e-4, 1.0, 1.0, 1.0, 1.0,
                0.0, 0.0, 1.0 / 3.0};
    return p;
}

static double maxabs(const double* a, size_t n) {
    double m = 0.0;
    for (size_t k = 0; k < n; ++k) {
        if (!isfinite(a[k])) return INFINITY;
        if (fabs(a[k]) > m) m = fabs(a[k]);
    }
    return m;
}

static int run_case(const char* name, params p, int perturbed, long steps) {
    const size_t n = (size_t)p.nx * p.ny;
    double* pop = malloc(27 * n * sizeof(double));
    double* f[5];
    for (int k = 0; k < 5; ++k) f[k] = malloc(n * sizeof(double));
    if (!pop || !f[0] || !f[1] || !f[2] || !f[3] || !f[4]) return 1;
    int rc;
    if (perturbed) {
        for (int j = 0; j < p.ny; ++j)
            for (int i = 0; i < p.nx; ++i) {
                const size_t q = (size_t)j * p.nx + i;
                const double h = (p.b - 0.5) + 0.8 * cos(2.0 * M_PI * i / p.nx);
                f[0][q] = 0.5 * (1.0 + tanh(2.0 * (h - j) / p.W));
                f[1][q] = 1e-4 * sin(2.0 * M_PI * i / p.nx);
                f[2][q] = -1e-4 * cos(2.0 * M_PI * j / p.ny);
                f[3][q] = 1.0 + 0.01 * sin(1.3 * i + 0.7 * j);
            }
        rc = orc_init_fields(&p, f[0], f[1], f[2], f[3], pop);
    } else {
        rc = orc_init_cold(&p, pop);
    }
    if (rc == 0) rc = orc_run(&p, pop, steps);
    if (rc == 0) rc = orc_macros(&p, pop, f[0], f[1], f[2], f[3], f[4]);
    double m = maxabs(pop, 27 * n);
    for (int k = 0; k < 5; ++k) {
        const double mk = maxabs(f[k], n);
        m = mk > m ? mk : m;
    }
    printf("%s: rc %d, max |value| %.6g\n", name, rc, m);
    for (int k = 0; k < 5; ++k) free(f[k]);
    free(pop);
    return rc != 0 || !isfinite(m);
}

int main(void) {
    int bad = 0;
    orc_set_threads(1);
    double P[81], Pi[81], w[9], F[9][9];
    int ex[9], ey[9];
    orc_tables(P, Pi, w, ex, ey);
    orc_build_F(0.03, -0.02, F);
    double in[9], out[9];
    for (int k = 0; k < 9; ++k) in[k] = w[k] * (0.5 + 0.01 * k);
    orc_collide_f_node(in, 0.5, 0.01, -0.02, 0.6, -0.8, 0.2, 0.02, 1.5, out);
    bad |= !isfinite(maxabs(out, 9));
    orc_collide_g_node(in, 0.34, 1.3, 0.01, -0.02, 1e-3, -2e-3, 3e-3, 1e-3, 1.2, out);
    bad |= !isfinite(maxabs(out, 9));
    orc_collide_h_node(in, 0.7, 0.01, -0.02, 1.3, out);
    bad |= !isfinite(maxabs(out, 9));
    printf("node maps: %s\n", bad ? "non-finite" : "ok");

    bad |= run_case("cold 32x16", base(32, 16, 8.0), 0, 60);
    params q = base(24, 12, 5.0);
    q.rho_b = 2.0; q.mu_a = 0.3; q.k_a = 0.05; q.n_waves = 2;
    bad |= run_case("perturbed 24x12, density ratio 2", q, 1, 40);
    params t = base(8, 4, 2.0);
    t.W = 1.5;
    bad |= run_case("tiny 8x4", t, 1, 20);
    return bad ? 1 : 0;
}
