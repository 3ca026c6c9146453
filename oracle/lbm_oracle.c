/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference of one time step of the coupled
 * central-moment lattice Boltzmann method of Elbousefi, Schupbach, Premnath
 * and Welch, "Thermocapillary convection in superimposed layers of
 * self-rewetting fluids" (arXiv 2210.07501).  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product path (the HIP library) never does, and the two share no code.
 *
 * The step follows the paper's order and notation, node by node:
 *   Sec. 4.1  conservative Allen-Cahn LBM for the order parameter (f)
 *   Sec. 4.2  pressure-based two-fluid LBM with surface-tension force (g)
 *   Sec. 4.3  energy-transport LBM for the temperature (h)
 * with the moment maps written out as the literal 9x9 matrices of App. B
 * (P and P^-1 as printed; F built from the binomial expansion that Sec. 4.1
 * states, F^-1 = F(-u)), the CSF force of Sec. 3 (Eq. eqn6 and its component
 * form), the quadratic surface-tension law Eq. (ST_SRF), the linear property
 * interpolation Eq. (eqn11) and the boundary schemes named in Sec. 5
 * (half-way bounce-back, anti-bounce-back, free-slip).
 *
 * Readings where the paper is silent or inconsistent (each also listed in the
 * design notes of the repository):
 *   - sharpening coefficient theta = +4 phi (1-phi) / W (Sec. 3 prints the
 *     opposite sign for phi_A = 0, phi_B = 1, which would anti-sharpen);
 *   - properties: X(phi) = X_a + phi (X_b - X_a), phi = 0 top fluid a,
 *     phi = 1 bottom fluid b; alpha = k / (rho c_p) with c_p = 1;
 *   - F row (22): binomial coefficients (-2 u_x u_y^2, -2 u_x^2 u_y), not the
 *     printed (-u_x u_y^2, -u_x^2 u_y);
 *   - the interface delta function 1.5 W |grad phi|^2 multiplies both force
 *     components (the component form in Sec. 3 drops the 1.5 W);
 *   - n = grad phi / sqrt(|grad phi|^2 + 1e-12) (regularised where grad phi
 *     vanishes, so that rounding noise in the bulk phases is not sharpened);
 *   - F_p = -grad(p* - rho c_s^2) uses p* = sum_a g_a of the current step;
 *   - curvature = isotropic divergence of n evaluated at the 8 neighbours;
 *   - stencil ghost rows: phi, p*, rho mirrored about the wall plane,
 *     T_ghost = 2 T_wall - T_adjacent;
 *   - anti-bounce-back wall temperature taken at the boundary node's column;
 *   - phi at the walls: specular (free-slip) reflection.
 *
 * Pins (tests/test_oracle_maps.py, test_oracle_physics.py, test_analytic.py)
 * cover every term: the forced central-moment relaxation of each collision
 * is checked moment by moment against Secs. 4.1-4.3 (the (1 - omega / 2)
 * factor of the shear modes included), and the T ghost rows by a vertical
 * interface meeting both walls in a linear temperature field, where the
 * wall rows must carry the same Marangoni force per sigma'(T) as the rows
 * between them.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, n_waves;
    double b;            /* thickness of bottom fluid b (phi = 1), cells   */
    double W, M_phi;     /* interface width, Allen-Cahn mobility           */
    double rho_a, rho_b, mu_a, mu_b, k_a, k_b;
    double sigma0, sigma_T, sigma_TT, T_ref;
    double T_h, dT, T_c; /* bottom wall T_h + dT cos(2 pi x / l), top T_c  */
    double Fx_ext, Fy_ext;
    double p0;           /* rest pressure (cold start)                     */
} orc_params;

/* D2Q9 velocity set (Sec. 4.1; last e_x entry taken from row 2 of P in
 * App. B, the printed e_x vector ends in 0 by a typo). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* D2Q9 weights; they are P^-1 applied to the rest raw moments
 * (1,0,0,1/3,1/3,0,0,0,1/9), which the test suite checks. */
static const double WGT[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double CS2 = 1.0 / 3.0;
/* regularisation of the unit normal where grad phi vanishes */
static const double EPS_N = 1e-6;

/* Moment order of the paper: (00,10,01,20,02,11,21,12,22). */
static const int MM[9] = {0, 1, 0, 2, 0, 1, 2, 1, 2};
static const int NN[9] = {0, 0, 1, 0, 2, 1, 1, 2, 2};

/* App. B, matrix P (raw moments from distributions), as printed. */
static const double PMAT[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 1, 0, 1, 0, 1, 1, 1, 1},
    {0, 0, 1, 0, 1, 1, 1, 1, 1},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 1, 1, 1, 1}};

/* App. B, matrix P^-1 (distributions from raw moments), as printed. */
static const double PINV[9][9] = {
    {1, 0, 0, -1, -1, 0, 0, 0, 1},
    {0, 0.5, 0, 0.5, 0, 0, 0, -0.5, -0.5},
    {0, 0, 0.5, 0, 0.5, 0, -0.5, 0, -0.5},
    {0, -0.5, 0, 0.5, 0, 0, 0, 0.5, -0.5},
    {0, 0, -0.5, 0, 0.5, 0, 0.5, 0, -0.5},
    {0, 0, 0, 0, 0, 0.25, 0.25, 0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, 0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, 0.25, -0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, -0.25, 0.25, 0.25}};

static double binom(int n, int k) {
    static const double C[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 2, 1}};
    return C[n][k];
}

/* F(u): kappa = F kappa', the binomial expansion of
 * (e_x - u_x)^m (e_y - u_y)^n over e_x^m' e_y^n' (Sec. 4.1). */
void orc_build_F(double ux, double uy, double F[9][9]) {
    const double px[3] = {1.0, -ux, ux * ux};   /* (-u_x)^k, k = 0, 1, 2 */
    const double py[3] = {1.0, -uy, uy * uy};
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            int m = MM[r], n = NN[r], mp = MM[c], np = NN[c];
            if (mp > m || np > n) { F[r][c] = 0.0; continue; }
            F[r][c] = binom(m, mp) * binom(n, np) * px[m - mp] * py[n - np];
        }
}

static void matvec(const double A[9][9], const double* x, double* y) {
    for (int r = 0; r < 9; ++r) {
        double s = 0.0;
        for (int c = 0; c < 9; ++c) s += A[r][c] * x[c];
        y[r] = s;
    }
}

/* Export the constant tables so that the tests can check them. */
void orc_tables(double* P, double* Pinv, double* w, int* ex, int* ey) {
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) { P[r * 9 + c] = PMAT[r][c]; Pinv[r * 9 + c] = PINV[r][c]; }
    for (int a = 0; a < 9; ++a) { w[a] = WGT[a]; ex[a] = EX[a]; ey[a] = EY[a]; }
}

/* ---- properties and surface tension ---------------------------------- */
static double interp(double phi, double xa, double xb) { return xa + phi * (xb - xa); }

/* Eq. (ST_SRF). */
static double sigma_of_T(const orc_params* p, double T) {
    double d = T - p->T_ref;
    return p->sigma0 + p->sigma_T * d + p->sigma_TT * d * d;
}

static double T_bottom(const orc_params* p, int i) {
    double l = (double)p->nx / (double)p->n_waves;
    return p->T_h + p->dT * cos(2.0 * M_PI * (double)i / l);
}

static int opposite(int a) {
    static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return OPP[a];
}
/* Direction with the same e_x and reversed e_y (specular reflection). */
static int mirror_y(int a) {
    static const int MIR[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
    return MIR[a];
}

#define POP(buf, d, a, j, i) (buf)[((((size_t)(d)) * 9 + (a)) * (size_t)ny + (j)) * (size_t)nx + (i)]

/* ---- node-wise collisions (App. B maps) --------------------------------- */

/* Sec. 4.1: collision of the phase-field distribution. */
static void collide_f(const double* f, double phi, double ux, double uy,
                      double nxv, double nyv, double theta, double M, double w_phi,
                      double* fout) {
    double kp[9], k[9], kt[9], ktp[9], F[9][9], Fi[9][9];
    matvec(PMAT, f, kp);
    orc_build_F(ux, uy, F);
    matvec(F, kp, k);
    double keq[9] = {phi, M * theta * nxv, M * theta * nyv, CS2 * phi, CS2 * phi,
                     0.0, 0.0, 0.0, CS2 * CS2 * phi};
    for (int r = 0; r < 9; ++r) {
        double w = (r == 1 || r == 2) ? w_phi : 1.0;
        kt[r] = k[r] + w * (keq[r] - k[r]);
    }
    orc_build_F(-ux, -uy, Fi);
    matvec(Fi, kt, ktp);
    matvec(PINV, ktp, fout);
}

/* Sec. 4.2: collision of the hydrodynamic distribution with sources. */
static void collide_g(const double* g, double p, double rho, double ux, double uy,
                      double Ftx, double Fty, double Fpx, double Fpy, double w_nu,
                      double* gout) {
    double ep[9], e[9], et[9], etp[9], F[9][9], Fi[9][9];
    matvec(PMAT, g, ep);
    orc_build_F(ux, uy, F);
    matvec(F, ep, e);
    double vphi = p - rho * CS2;      /* varphi(rho) = p - rho c_s^2 */
    double ux2 = ux * ux, uy2 = uy * uy;
    double eq[9];
    eq[0] = p;
    eq[1] = -vphi * ux;
    eq[2] = -vphi * uy;
    eq[3] = p * CS2 + vphi * ux2;
    eq[4] = p * CS2 + vphi * uy2;
    eq[5] = vphi * ux * uy;
    eq[6] = -vphi * (ux2 + CS2) * uy;
    eq[7] = -vphi * (uy2 + CS2) * ux;
    eq[8] = CS2 * CS2 * CS2 * rho + vphi * (ux2 + CS2) * (uy2 + CS2);
    double G = Fpx * ux + Fpy * uy;   /* Gamma_00^p */
    double s[9];
    s[0] = G;
    s[1] = CS2 * Ftx - ux * G;
    s[2] = CS2 * Fty - uy * G;
    s[3] = 2.0 * CS2 * Fpx * ux + (ux2 + CS2) * G;
    s[4] = 2.0 * CS2 * Fpy * uy + (uy2 + CS2) * G;
    s[5] = CS2 * (Fpx * uy + Fpy * ux) + ux * uy * G;
    s[6] = 0.0;
    s[7] = 0.0;
    s[8] = 0.0;
    /* trace / deviator split of the second-order diagonal moments */
    double e2s = e[3] + e[4], e2d = e[3] - e[4];
    double q2s = eq[3] + eq[4], q2d = eq[3] - eq[4];
    double s2s = s[3] + s[4], s2d = s[3] - s[4];
    /* relaxation rates: shear (2d, 11) at omega_nu, everything else 1 */
    for (int r = 0; r < 9; ++r) {
        double w = (r == 5) ? w_nu : 1.0;
        et[r] = e[r] + w * (eq[r] - e[r]) + (1.0 - 0.5 * w) * s[r];
    }
    double t2s = e2s + 1.0 * (q2s - e2s) + (1.0 - 0.5) * s2s;
    double t2d = e2d + w_nu * (q2d - e2d) + (1.0 - 0.5 * w_nu) * s2d;
    et[3] = 0.5 * (t2s + t2d);
    et[4] = 0.5 * (t2s - t2d);
    orc_build_F(-ux, -uy, Fi);
    matvec(Fi, et, etp);
    matvec(PINV, etp, gout);
}

/* Sec. 4.3: collision of the energy distribution. */
static void collide_h(const double* h, double T, double ux, double uy, double w_T,
                      double* hout) {
    double cp[9], c[9], ct[9], ctp[9], F[9][9], Fi[9][9];
    matvec(PMAT, h, cp);
    orc_build_F(ux, uy, F);
    matvec(F, cp, c);
    double ceq[9] = {T, 0.0, 0.0, CS2 * T, CS2 * T, 0.0, 0.0, 0.0, CS2 * CS2 * T};
    for (int r = 0; r < 9; ++r) {
        double w = (r == 1 || r == 2) ? w_T : 1.0;
        ct[r] = c[r] + w * (ceq[r] - c[r]);
    }
    orc_build_F(-ux, -uy, Fi);
    matvec(Fi, ct, ctp);
    matvec(PINV, ctp, hout);
}

/* Exported single-node maps, for the round-trip and invariant tests. */
void orc_collide_f_node(const double* f, double phi, double ux, double uy, double nxv,
                        double nyv, double theta, double M, double w_phi, double* out) {
    collide_f(f, phi, ux, uy, nxv, nyv, theta, M, w_phi, out);
}
void orc_collide_g_node(const double* g, double p, double rho, double ux, double uy,
                        double Ftx, double Fty, double Fpx, double Fpy, double w_nu,
                        double* out) {
    collide_g(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, w_nu, out);
}
void orc_collide_h_node(const double* h, double T, double ux, double uy, double w_T,
                        double* out) {
    collide_h(h, T, ux, uy, w_T, out);
}

/* ---- macroscopic fields and forces --------------------------------------- */

typedef struct {
    double *phi, *T, *ps, *rho;      /* padded: phi 2 ghost rows, others 1   */
    double *jx, *jy;                 /* unpadded                             */
    double *gx, *gy, *nxf, *nyf;     /* grad phi and normal, 1 ghost row     */
} work_t;

static int work_alloc(work_t* w, int nx, int ny) {
    size_t n2 = (size_t)nx * (ny + 4), n1 = (size_t)nx * (ny + 2), n0 = (size_t)nx * ny;
    w->phi = malloc(n2 * sizeof(double));
    w->T = malloc(n1 * sizeof(double));
    w->ps = malloc(n1 * sizeof(double));
    w->rho = malloc(n1 * sizeof(double));
    w->gx = malloc(n1 * sizeof(double));
    w->gy = malloc(n1 * sizeof(double));
    w->nxf = malloc(n1 * sizeof(double));
    w->nyf = malloc(n1 * sizeof(double));
    w->jx = malloc(n0 * sizeof(double));
    w->jy = malloc(n0 * sizeof(double));
    return w->phi && w->T && w->ps && w->rho && w->gx && w->gy && w->nxf && w->nyf &&
           w->jx && w->jy;
}
static void work_free(work_t* w) {
    free(w->phi); free(w->T); free(w->ps); free(w->rho); free(w->gx); free(w->gy);
    free(w->nxf); free(w->nyf); free(w->jx); free(w->jy);
}

/* padded row index helpers: PH rows -2..ny+1, P1 rows -1..ny */
#define PH(w, j, i) (w)->phi[((size_t)((j) + 2)) * nx + (i)]
#define P1(arr, j, i) (arr)[((size_t)((j) + 1)) * nx + (i)]

static int wrap(int i, int nx) { int r = i % nx; return r < 0 ? r + nx : r; }

/* Isotropic first derivative (Sec. 3, isotropic finite differences):
 * d/dx psi = (1/c_s^2) sum_a w_a e_ax psi(x + e_a), same for y. */
#define ISO_GRAD(ACC, jj, ii, OUTX, OUTY)                                        \
    do {                                                                         \
        double sx_ = 0.0, sy_ = 0.0;                                             \
        for (int a_ = 1; a_ < 9; ++a_) {                                         \
            double v_ = ACC((jj) + EY[a_], wrap((ii) + EX[a_], nx));             \
            sx_ += WGT[a_] * EX[a_] * v_;                                        \
            sy_ += WGT[a_] * EY[a_] * v_;                                        \
        }                                                                        \
        OUTX = sx_ / CS2;                                                        \
        OUTY = sy_ / CS2;                                                        \
    } while (0)

/* Step 1-3: moments of the streamed populations, properties, ghost rows. */
static void fill_macros(const orc_params* P, const double* pop, work_t* w) {
    const int nx = P->nx, ny = P->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double phi = 0, T = 0, ps = 0, jx = 0, jy = 0;
            for (int a = 0; a < 9; ++a) {
                double fv = POP(pop, 0, a, j, i), gv = POP(pop, 1, a, j, i), hv = POP(pop, 2, a, j, i);
                phi += fv;
                ps += gv;
                T += hv;
                jx += gv * EX[a];
                jy += gv * EY[a];
            }
            PH(w, j, i) = phi;
            P1(w->T, j, i) = T;
            P1(w->ps, j, i) = ps;
            P1(w->rho, j, i) = interp(phi, P->rho_a, P->rho_b);
            w->jx[(size_t)j * nx + i] = jx;
            w->jy[(size_t)j * nx + i] = jy;
        }
    /* ghost rows: mirror about the wall planes y = -1/2 and y = ny - 1/2 */
    for (int i = 0; i < nx; ++i) {
        PH(w, -1, i) = PH(w, 0, i);
        PH(w, -2, i) = PH(w, 1, i);
        PH(w, ny, i) = PH(w, ny - 1, i);
        PH(w, ny + 1, i) = PH(w, ny - 2, i);
        P1(w->ps, -1, i) = P1(w->ps, 0, i);
        P1(w->ps, ny, i) = P1(w->ps, ny - 1, i);
        P1(w->rho, -1, i) = P1(w->rho, 0, i);
        P1(w->rho, ny, i) = P1(w->rho, ny - 1, i);
        P1(w->T, -1, i) = 2.0 * T_bottom(P, i) - P1(w->T, 0, i);
        P1(w->T, ny, i) = 2.0 * P->T_c - P1(w->T, ny - 1, i);
    }
    /* grad phi and unit normal on rows -1..ny */
#define ACC_PHI(jj, ii) PH(w, jj, ii)
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double gx, gy;
            ISO_GRAD(ACC_PHI, j, i, gx, gy);
            double den = sqrt(gx * gx + gy * gy + EPS_N * EPS_N);
            P1(w->gx, j, i) = gx;
            P1(w->gy, j, i) = gy;
            P1(w->nxf, j, i) = gx / den;
            P1(w->nyf, j, i) = gy / den;
        }
#undef ACC_PHI
}

typedef struct {
    double phi, T, rho, p, ux, uy, Ftx, Fty, Fpx, Fpy, nx, ny, theta, w_nu, w_T;
} node_state;

/* Steps 4-6 at node (i, j): stencils, forces, corrected velocity and pressure. */
static node_state node_macros(const orc_params* P, const work_t* w, int i, int j) {
    const int nx = P->nx;
    node_state s;
    s.phi = PH(w, j, i);
    s.T = P1(w->T, j, i);
    s.rho = P1(w->rho, j, i);
    double ps = P1(w->ps, j, i);
    double gx = P1(w->gx, j, i), gy = P1(w->gy, j, i);
    double g2 = gx * gx + gy * gy;
    s.nx = P1(w->nxf, j, i);
    s.ny = P1(w->nyf, j, i);
    /* curvature kappa = div n (isotropic stencil over neighbour normals) */
    double dnx_dx, dnx_dy, dny_dx, dny_dy;
#define ACC_NX(jj, ii) P1(w->nxf, jj, ii)
#define ACC_NY(jj, ii) P1(w->nyf, jj, ii)
    ISO_GRAD(ACC_NX, j, i, dnx_dx, dnx_dy);
    ISO_GRAD(ACC_NY, j, i, dny_dx, dny_dy);
    (void)dnx_dy; (void)dny_dx;
    double curv = dnx_dx + dny_dy;
    /* surface tension and its isotropic gradient */
    double sig = sigma_of_T(P, s.T);
    double dsx, dsy;
#define ACC_SIG(jj, ii) sigma_of_T(P, P1(w->T, jj, ii))
    ISO_GRAD(ACC_SIG, j, i, dsx, dsy);
    /* pressure force F_p = -grad(p* - rho c_s^2) */
    double dvx, dvy;
#define ACC_VP(jj, ii) (P1(w->ps, jj, ii) - P1(w->rho, jj, ii) * CS2)
    ISO_GRAD(ACC_VP, j, i, dvx, dvy);
#undef ACC_NX
#undef ACC_NY
#undef ACC_SIG
#undef ACC_VP
    /* CSF force, Sec. 3: delta_s [ -sigma kappa n + (I - n n) grad sigma ] */
    double delta_s = 1.5 * P->W * g2;
    double Fsx = delta_s * (-sig * curv * s.nx + (1.0 - s.nx * s.nx) * dsx - s.nx * s.ny * dsy);
    double Fsy = delta_s * (-sig * curv * s.ny + (1.0 - s.ny * s.ny) * dsy - s.nx * s.ny * dsx);
    s.Ftx = Fsx + P->Fx_ext;
    s.Fty = Fsy + P->Fy_ext;
    s.Fpx = -dvx;
    s.Fpy = -dvy;
    /* Sec. 4.2 macroscopic update: rho c_s^2 u = sum g e + c_s^2 F_t / 2,
     * p = sum g + F_p . u / 2 */
    double jx = w->jx[(size_t)j * nx + i], jy = w->jy[(size_t)j * nx + i];
    s.ux = (jx + 0.5 * CS2 * s.Ftx) / (s.rho * CS2);
    s.uy = (jy + 0.5 * CS2 * s.Fty) / (s.rho * CS2);
    s.p = ps + 0.5 * (s.Fpx * s.ux + s.Fpy * s.uy);
    /* relaxation rates from the local properties */
    double mu = interp(s.phi, P->mu_a, P->mu_b);
    double kc = interp(s.phi, P->k_a, P->k_b);
    double nu = mu / s.rho, alpha = kc / s.rho;
    s.w_nu = 1.0 / (nu / CS2 + 0.5);
    s.w_T = 1.0 / (alpha / CS2 + 0.5);
    s.theta = 4.0 * s.phi * (1.0 - s.phi) / P->W;
    return s;
}

/* Macroscopic fields of the current state (corrected u and p). */
int orc_macros(const orc_params* P, const double* pop, double* phi, double* ux,
               double* uy, double* T, double* p) {
    const int nx = P->nx, ny = P->ny;
    work_t w;
    if (!work_alloc(&w, nx, ny)) { work_free(&w); return -1; }
    fill_macros(P, pop, &w);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            node_state s = node_macros(P, &w, i, j);
            size_t q = (size_t)j * nx + i;
            if (phi) phi[q] = s.phi;
            if (ux) ux[q] = s.ux;
            if (uy) uy[q] = s.uy;
            if (T) T[q] = s.T;
            if (p) p[q] = s.p;
        }
    work_free(&w);
    return 0;
}

/* One time step: collide every node (Secs. 4.1-4.3) then stream with the
 * wall schemes of Sec. 5.  pop_in and pop_out must not alias. */
int orc_step(const orc_params* P, const double* pop_in, double* pop_out) {
    const int nx = P->nx, ny = P->ny;
    const double w_phi = 1.0 / (P->M_phi / CS2 + 0.5);
    work_t w;
    if (!work_alloc(&w, nx, ny)) { work_free(&w); return -1; }
    double* post = malloc((size_t)27 * nx * ny * sizeof(double));
    if (!post) { work_free(&w); return -1; }
    fill_macros(P, pop_in, &w);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            node_state s = node_macros(P, &w, i, j);
            double fin[9], gin[9], hin[9], fo[9], go[9], ho[9];
            for (int a = 0; a < 9; ++a) {
                fin[a] = POP(pop_in, 0, a, j, i);
                gin[a] = POP(pop_in, 1, a, j, i);
                hin[a] = POP(pop_in, 2, a, j, i);
            }
            collide_f(fin, s.phi, s.ux, s.uy, s.nx, s.ny, s.theta, P->M_phi, w_phi, fo);
            collide_g(gin, s.p, s.rho, s.ux, s.uy, s.Ftx, s.Fty, s.Fpx, s.Fpy, s.w_nu, go);
            collide_h(hin, s.T, s.ux, s.uy, s.w_T, ho);
            for (int a = 0; a < 9; ++a) {
                POP(post, 0, a, j, i) = fo[a];
                POP(post, 1, a, j, i) = go[a];
                POP(post, 2, a, j, i) = ho[a];
            }
        }
    /* streaming: x_new = x_old + e_a; links through a wall plane reflect */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int a = 0; a < 9; ++a) {
                int js = j - EY[a], is = wrap(i - EX[a], nx);
                if (js >= 0 && js < ny) {
                    for (int d = 0; d < 3; ++d) POP(pop_out, d, a, j, i) = POP(post, d, a, js, is);
                } else {
                    double Tw = (js < 0) ? T_bottom(P, i) : P->T_c;
                    /* f: free-slip (specular) reflection */
                    POP(pop_out, 0, a, j, i) = POP(post, 0, mirror_y(a), j, is);
                    /* g: half-way bounce-back (no slip) */
                    POP(pop_out, 1, a, j, i) = POP(post, 1, opposite(a), j, i);
                    /* h: anti-bounce-back (Dirichlet temperature) */
                    POP(pop_out, 2, a, j, i) = -POP(post, 2, opposite(a), j, i) + 2.0 * WGT[a] * Tw;
                }
            }
    free(post);
    work_free(&w);
    return 0;
}

/* n steps with internal double buffering; the result is left in pop. */
int orc_run(const orc_params* P, double* pop, long nsteps) {
    size_t n = (size_t)27 * P->nx * P->ny;
    double* tmp = malloc(n * sizeof(double));
    if (!tmp) return -1;
    for (long s = 0; s < nsteps; ++s) {
        if (orc_step(P, pop, tmp)) { free(tmp); return -1; }
        memcpy(pop, tmp, n * sizeof(double));
    }
    free(tmp);
    return 0;
}

/* Populations at equilibrium for given (phi, u, T) and rest pressure p0:
 * f = P^-1 F(-u) kappa^eq (without the sharpening flux), g = P^-1 F(-u) eta^eq,
 * h = P^-1 F(-u) chi^eq.  The paper does not state an initial state. */
int orc_init_fields(const orc_params* P, const double* phi, const double* ux,
                    const double* uy, const double* T, double* pop) {
    const int nx = P->nx, ny = P->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t q = (size_t)j * nx + i;
            double ph = phi[q], vx = ux[q], vy = uy[q], Tq = T[q];
            double rho = interp(ph, P->rho_a, P->rho_b), p = P->p0;
            double vphi = p - rho * CS2, vx2 = vx * vx, vy2 = vy * vy;
            double keq[9] = {ph, 0, 0, CS2 * ph, CS2 * ph, 0, 0, 0, CS2 * CS2 * ph};
            double eeq[9] = {p, -vphi * vx, -vphi * vy, p * CS2 + vphi * vx2,
                             p * CS2 + vphi * vy2, vphi * vx * vy, -vphi * (vx2 + CS2) * vy,
                             -vphi * (vy2 + CS2) * vx,
                             CS2 * CS2 * CS2 * rho + vphi * (vx2 + CS2) * (vy2 + CS2)};
            double ceq[9] = {Tq, 0, 0, CS2 * Tq, CS2 * Tq, 0, 0, 0, CS2 * CS2 * Tq};
            double Fi[9][9], r[9], o[9];
            orc_build_F(-vx, -vy, Fi);
            matvec(Fi, keq, r); matvec(PINV, r, o);
            for (int a = 0; a < 9; ++a) POP(pop, 0, a, j, i) = o[a];
            matvec(Fi, eeq, r); matvec(PINV, r, o);
            for (int a = 0; a < 9; ++a) POP(pop, 1, a, j, i) = o[a];
            matvec(Fi, ceq, r); matvec(PINV, r, o);
            for (int a = 0; a < 9; ++a) POP(pop, 2, a, j, i) = o[a];
        }
    return 0;
}

/* Cold-start fields: fluid at rest, tanh interface centred on the plane
 * y = b - 1/2 (bottom fluid phi = 1), temperature linear between the walls. */
void orc_cold_fields(const orc_params* P, double* phi, double* ux, double* uy, double* T) {
    const int nx = P->nx, ny = P->ny;
    double yint = P->b - 0.5;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t q = (size_t)j * nx + i;
            phi[q] = 0.5 * (1.0 + tanh(2.0 * (yint - (double)j) / P->W));
            ux[q] = 0.0;
            uy[q] = 0.0;
            double Tb = T_bottom(P, i);
            T[q] = Tb + (P->T_c - Tb) * ((double)j + 0.5) / (double)ny;
        }
}

int orc_init_cold(const orc_params* P, double* pop) {
    size_t n = (size_t)P->nx * P->ny;
    double* buf = malloc(4 * n * sizeof(double));
    if (!buf) return -1;
    orc_cold_fields(P, buf, buf + n, buf + 2 * n, buf + 3 * n);
    int rc = orc_init_fields(P, buf, buf + n, buf + 2 * n, buf + 3 * n, pop);
    free(buf);
    return rc;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later steps (timing only; the result does not depend on it). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
