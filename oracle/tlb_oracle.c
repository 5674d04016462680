/*
 * tlb_oracle.c -- plain FP64 CPU oracle of the ternary phase-field lattice
 * Boltzmann step with the ternary wetting boundary scheme (Liang et al.,
 * arXiv:1710.09534).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the GPU
 * library or its binding.
 *
 * One step is a sequence of full-field loops, each writing its own array:
 *   S1  moments c_i (Eq. 13a), c3 (Eq. 3), rho, nu (Eqs. 14-15), tau_g (Eq. 18b)
 *   S2  wetting ghosts at solid links (Eq. 42)
 *   S3  Laplacian of c_i (Eq. 20b) with those ghosts
 *   S4  chemical potentials (Eq. 8)
 *   S5  gradients of c_i and rho, Laplacian of mu_i, symmetric ghosts (Eq. 43)
 *   S6  F_s (potential form), body force G, velocity (Eq. 13b)
 *   S7  interfacial force F_a (Eq. 12)
 *   S8  pressure (Eq. 13c)
 *   S9  Euler time derivative of c_i u (Eq. 19)
 *   S10 equilibria (Eqs. 2, 4) and source terms (Eq. 11)
 *   S11 BGK collision (Eq. 45)
 *   S11b post-collision populations of velocity boundary nodes by the
 *       non-equilibrium extrapolation scheme (Eqs. 51-53)
 *   S12 streaming with half-way bounce-back (Eq. 44) and, for a moving wall,
 *       the momentum correction of the bounced populations.
 * A velocity boundary node x_u shows, to every stencil and to its own
 * equilibria, the macroscopic values of the fluid node x_f directly inside
 * it (the interpolation chi(x_u) = chi(x_f) stated with Eq. 53); only the
 * velocity is the prescribed one.
 * Built with -O2 -ffp-contract=off; OpenMP only splits rows of a loop, so
 * results do not depend on the thread count.
 */
#include "tlb_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- lattice */
/* D2Q9, Eq. 10: rest, four axis links at angles (k-1)pi/2, four diagonal
 * links of length sqrt(2) at angles (k-5)pi/2 + pi/4. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 with c = 1 */

static char g_err[512];
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char* orc_last_error(void) { return g_err; }

void orc_lattice(int ex[9], int ey[9], double w[9], int opp[9]) {
    for (int k = 0; k < 9; ++k) {
        ex[k] = EX[k];
        ey[k] = EY[k];
        w[k] = W[k];
        opp[k] = OPP[k];
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------- parameters */
/* lambda_i from the pairwise surface tensions (Eq. 7), lambda_T from
 * 3/lambda_T = sum 1/lambda_i (Eq. 9), M_i = M0/lambda_i (Eq. 12), and
 * eta_i from M_i = eta c_s^2 (tau_i - 1/2) (Eq. 18a).  With unequal
 * lambda_1, lambda_2 one scalar eta cannot satisfy both Eq. 12 and Eq. 18a,
 * so eta is solved per component. */
int orc_params(const orc_fluid* fl, orc_derived* out) {
    double l1 = fl->sigma12 + fl->sigma13 - fl->sigma23;
    double l2 = fl->sigma12 + fl->sigma23 - fl->sigma13;
    double l3 = fl->sigma13 + fl->sigma23 - fl->sigma12;
    out->lambda[0] = l1;
    out->lambda[1] = l2;
    out->lambda[2] = l3;
    out->lambdaT = 3.0 / (1.0 / l1 + 1.0 / l2 + 1.0 / l3);
    out->M[0] = fl->M0 / l1;
    out->M[1] = fl->M0 / l2;
    out->eta[0] = out->M[0] / (CS2 * (fl->tau1 - 0.5));
    out->eta[1] = out->M[1] / (CS2 * (fl->tau2 - 0.5));
    /* lambda_i > 0 (M_i = M0/lambda_i and Eq. 9 need it); the condition
     * lambda_i > lambda_T/2 is stated for the energy with lambda = 0, so it
     * is required only then */
    if (!(fl->lambda >= 0.0)) return -1;
    for (int i = 0; i < 3; ++i) {
        if (!(out->lambda[i] > 0.0)) return -1;
        if (fl->lambda == 0.0 && !(out->lambda[i] > 0.5 * out->lambdaT)) return -1;
    }
    return 0;
}

/* Eq. 39 solved for theta12: sigma12 cos12 = sigma13 cos13 - sigma23 cos23 */
int orc_cos12(const orc_fluid* fl, double theta13_deg, double theta23_deg, double* cos12) {
    const double d2r = acos(-1.0) / 180.0;
    double c13 = cos(theta13_deg * d2r);
    double c23 = cos(theta23_deg * d2r);
    double c12 = (fl->sigma13 * c13 - fl->sigma23 * c23) / fl->sigma12;
    *cos12 = c12;
    return fabs(c12) <= 1.0 ? 0 : -1;
}

/* ---------------------------------------------------------------- pointwise */
/* Eq. 42: ghost order parameters seen across a solid link from fluid node
 * x_f, with the wall value taken as c(x_f) and dx = 1. */
void orc_wetting_ghost(double D, double cos12, double cos13, double cos23,
                       double c1, double c2, double out[3]) {
    double c3 = 1.0 - c1 - c2;
    double h1 = cos13 * c1 * c3 + cos12 * c1 * c2;
    double h2 = -cos12 * c1 * c2 + cos23 * c2 * c3;
    double h3 = -cos23 * c2 * c3 - cos13 * c1 * c3;
    out[0] = c1 + (4.0 / D) * h1;
    out[1] = c2 + (4.0 / D) * h2;
    out[2] = c3 + (4.0 / D) * h3;
}

/* Eq. 8 (bulk energy Eq. 5 with lambda = 0), i = 1, 2, 3, plus, for
 * lambda > 0, the part of Eq. 6 that comes from the lambda c1^2 c2^2 c3^2 term
 * of Eq. 5: with dP/dc_i = 2 lambda c_i c_j^2 c_k^2 ({i,j,k} = {1,2,3}),
 * (4 lambda_T / D) sum_{j != i} (dP/dc_i - dP/dc_j) / lambda_j. */
void orc_chem_potential(const orc_fluid* fl, double c1, double c2,
                        double lap1, double lap2, double lap3, double mu[3]) {
    orc_derived d;
    orc_params(fl, &d);
    double c3 = 1.0 - c1 - c2;
    double c[3] = {c1, c2, c3};
    double lap[3] = {lap1, lap2, lap3};
    double D = fl->D;
    for (int i = 0; i < 3; ++i) {
        double bulk = d.lambda[i] * c[i] * (1.0 - c[i]) * (1.0 - 2.0 * c[i])
                    - 2.0 * d.lambdaT * c1 * c2 * (1.0 - c1 - c2);
        mu[i] = (12.0 / D) * bulk - 0.75 * D * d.lambda[i] * lap[i];
    }
    if (fl->lambda != 0.0) {
        double dP[3];
        for (int i = 0; i < 3; ++i) {
            double prod = 1.0;
            for (int j = 0; j < 3; ++j)
                if (j != i) prod *= c[j] * c[j];
            dP[i] = 2.0 * fl->lambda * c[i] * prod;
        }
        for (int i = 0; i < 3; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j)
                if (j != i) acc += (dP[i] - dP[j]) / d.lambda[j];
            mu[i] += 4.0 * d.lambdaT / D * acc;
        }
    }
}

/* s_k(u) of Eq. 4 */
static double s_k(int k, double ux, double uy) {
    double eu = EX[k] * ux + EY[k] * uy;
    double uu = ux * ux + uy * uy;
    return W[k] * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

void orc_equilibria(double c1, double c2, double eta1, double eta2,
                    double mu1, double mu2, double rho, double p,
                    double ux, double uy,
                    double feq1[9], double feq2[9], double geq[9]) {
    for (int k = 0; k < 9; ++k) {
        double eu = EX[k] * ux + EY[k] * uy;
        if (k == 0) {
            /* Eq. 2a, k = 0 */
            feq1[k] = c1 + (W[k] - 1.0) * eta1 * mu1;
            feq2[k] = c2 + (W[k] - 1.0) * eta2 * mu2;
            /* Eq. 2b, k = 0 */
            geq[k] = p / CS2 * (W[k] - 1.0) + rho * s_k(k, ux, uy);
        } else {
            feq1[k] = W[k] * eta1 * mu1 + W[k] * c1 * eu / CS2;
            feq2[k] = W[k] * eta2 * mu2 + W[k] * c2 * eu / CS2;
            geq[k] = p / CS2 * W[k] + rho * s_k(k, ux, uy);
        }
    }
}

/* Eq. 11a with dt(c_i u) = D_i, and Eq. 11b as printed: the F_a term stands
 * outside the (1 - 1/(2 tau_g)) factor. */
void orc_sources(double tau1, double tau2, double taug,
                 double d1x, double d1y, double d2x, double d2y,
                 double ux, double uy, double grx, double gry,
                 double fx, double fy, double fax, double fay,
                 double F1[9], double F2[9], double G[9]) {
    for (int k = 0; k < 9; ++k) {
        double ed1 = EX[k] * d1x + EY[k] * d1y;
        double ed2 = EX[k] * d2x + EY[k] * d2y;
        F1[k] = (1.0 - 1.0 / (2.0 * tau1)) * W[k] * ed1 / CS2;
        F2[k] = (1.0 - 1.0 / (2.0 * tau2)) * W[k] * ed2 / CS2;
        double sk = s_k(k, ux, uy);
        double ax = EX[k] - ux, ay = EY[k] - uy;
        double bx = sk * grx + (sk + W[k]) * fx / CS2;
        double by = sk * gry + (sk + W[k]) * fy / CS2;
        double efa = EX[k] * fax + EY[k] * fay;
        G[k] = (1.0 - 1.0 / (2.0 * taug)) * (ax * bx + ay * by) + W[k] * efa / CS2;
    }
}

/* ---------------------------------------------------------------- lattice state */
typedef struct {
    double cos12, cos13, cos23;
    double uw[2];
    int kind;     /* ORC_WALL or ORC_VELOCITY */
} mat_t;

struct orc_sim {
    int nx, ny, px, py;
    long n;
    orc_fluid fl;
    orc_derived d;
    uint8_t* mat;
    int nmat;
    mat_t* mats;
    /* per node: 0 fluid, 1 wall, 2 velocity boundary; inner[i] is the fluid
     * node directly inside velocity boundary node i (else -1) */
    uint8_t* cls;
    long* inner;
    int inited;
    /* state: populations f(x,t) after streaming, and history at t-1 */
    double *f1[9], *f2[9], *g[9];
    double *c1o, *c2o, *uxo, *uyo;
    /* one array per intermediate */
    double *c1, *c2, *c3, *rho, *nu, *taug;
    double *lc1, *lc2, *lc3;
    double *mu1, *mu2, *mu3;
    double *gc1x, *gc1y, *gc2x, *gc2y, *gc3x, *gc3y, *grx, *gry;
    double *lmu1, *lmu2;
    double *fsx, *fsy, *gbx, *gby, *ux, *uy, *fax, *fay, *p;
    double *d1x, *d1y, *d2x, *d2y;
    double *fe1[9], *fe2[9], *ge[9];
    double *F1[9], *F2[9], *Gk[9];
    double *fp1[9], *fp2[9], *gp[9];
};

static double* alloc_field(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

/* neighbour of (x,y) along e_k with periodic wrap; -1 if it leaves a
 * non-periodic domain */
static long nbr(const orc_sim* s, int x, int y, int k) {
    int xn = x + EX[k], yn = y + EY[k];
    if (xn < 0 || xn >= s->nx) {
        if (!s->px) return -1;
        xn = (xn + s->nx) % s->nx;
    }
    if (yn < 0 || yn >= s->ny) {
        if (!s->py) return -1;
        yn = (yn + s->ny) % s->ny;
    }
    return (long)yn * s->nx + xn;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    double** all[] = {&s->c1o, &s->c2o, &s->uxo, &s->uyo, &s->c1, &s->c2, &s->c3, &s->rho,
                      &s->nu, &s->taug, &s->lc1, &s->lc2, &s->lc3, &s->mu1, &s->mu2, &s->mu3,
                      &s->gc1x, &s->gc1y, &s->gc2x, &s->gc2y, &s->gc3x, &s->gc3y, &s->grx,
                      &s->gry, &s->lmu1, &s->lmu2, &s->fsx, &s->fsy, &s->gbx, &s->gby,
                      &s->ux, &s->uy, &s->fax, &s->fay, &s->p, &s->d1x, &s->d1y, &s->d2x,
                      &s->d2y};
    for (size_t i = 0; i < sizeof all / sizeof all[0]; ++i) free(*all[i]);
    for (int k = 0; k < 9; ++k) {
        free(s->f1[k]); free(s->f2[k]); free(s->g[k]);
        free(s->fe1[k]); free(s->fe2[k]); free(s->ge[k]);
        free(s->F1[k]); free(s->F2[k]); free(s->Gk[k]);
        free(s->fp1[k]); free(s->fp2[k]); free(s->gp[k]);
    }
    free(s->mat);
    free(s->mats);
    free(s->cls);
    free(s->inner);
    free(s);
}

int orc_create(int nx, int ny, const orc_fluid* fl, int periodic_x, int periodic_y,
               const uint8_t* material, const orc_material* mats, int n_mats,
               orc_sim** out) {
    *out = NULL;
    if (nx < 3 || ny < 3 || !fl || !material || n_mats < 0 || (n_mats > 0 && !mats)) {
        set_err("invalid sizes or null pointer");
        return -1;
    }
    orc_derived d;
    if (fl->D <= 0 || fl->M0 <= 0 || fl->tau1 <= 0.5 || fl->tau2 <= 0.5) {
        set_err("D, M0 must be > 0 and tau_i > 1/2");
        return -2;
    }
    for (int i = 0; i < 3; ++i)
        if (!(fl->rho[i] > 0) || !(fl->nu[i] > 0)) {
            set_err("densities and viscosities must be > 0");
            return -2;
        }
    if (orc_params(fl, &d) != 0) {
        set_err("surface tensions violate lambda_i > 0 or lambda_i > lambda_T/2");
        return -2;
    }
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->nx = nx;
    s->ny = ny;
    s->px = periodic_x != 0;
    s->py = periodic_y != 0;
    s->n = (long)nx * ny;
    s->fl = *fl;
    s->d = d;
    s->nmat = n_mats;
    s->mats = (mat_t*)calloc((size_t)(n_mats > 0 ? n_mats : 1), sizeof(mat_t));
    const double d2r = acos(-1.0) / 180.0;
    for (int m = 0; m < n_mats; ++m) {
        double c12 = 0.0;
        if (mats[m].kind != ORC_WALL && mats[m].kind != ORC_VELOCITY) {
            set_err("unknown material kind");
            orc_destroy(s);
            return -1;
        }
        s->mats[m].kind = mats[m].kind;
        s->mats[m].uw[0] = mats[m].wall_u[0];
        s->mats[m].uw[1] = mats[m].wall_u[1];
        if (mats[m].kind == ORC_VELOCITY) continue;
        if (orc_cos12(fl, mats[m].theta13_deg, mats[m].theta23_deg, &c12) != 0) {
            set_err("contact angles give |cos theta12| > 1 (Eq. 39)");
            orc_destroy(s);
            return -2;
        }
        s->mats[m].cos12 = c12;
        s->mats[m].cos13 = cos(mats[m].theta13_deg * d2r);
        s->mats[m].cos23 = cos(mats[m].theta23_deg * d2r);
    }
    s->mat = (uint8_t*)malloc((size_t)s->n);
    memcpy(s->mat, material, (size_t)s->n);
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i] > n_mats) {
            set_err("material id exceeds the material table");
            orc_destroy(s);
            return -1;
        }
    }
    s->cls = (uint8_t*)malloc((size_t)s->n);
    s->inner = (long*)malloc((size_t)s->n * sizeof(long));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            s->inner[i] = -1;
            if (!s->mat[i]) { s->cls[i] = 0; continue; }
            if (s->mats[s->mat[i] - 1].kind == ORC_WALL) { s->cls[i] = 1; continue; }
            /* velocity boundary node: bottom or top row of a y-bounded lattice */
            s->cls[i] = 2;
            if (s->py || (y != 0 && y != ny - 1)) {
                set_err("velocity boundary nodes must lie in the bottom or top row of a "
                        "lattice that is not periodic in y");
                orc_destroy(s);
                return -1;
            }
            s->inner[i] = (long)(y == 0 ? 1 : ny - 2) * nx + x;
        }
    for (long i = 0; i < s->n; ++i)
        if (s->cls[i] == 2 && s->mat[s->inner[i]]) {
            set_err("the node inside a velocity boundary node must be fluid");
            orc_destroy(s);
            return -1;
        }
    /* a fluid node may not touch the edge of a non-periodic direction */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (s->mat[(long)y * nx + x]) continue;
            for (int k = 1; k < 9; ++k)
                if (nbr(s, x, y, k) < 0) {
                    set_err("fluid node on the edge of a non-periodic direction");
                    orc_destroy(s);
                    return -1;
                }
        }
    long n = s->n;
    double** all[] = {&s->c1o, &s->c2o, &s->uxo, &s->uyo, &s->c1, &s->c2, &s->c3, &s->rho,
                      &s->nu, &s->taug, &s->lc1, &s->lc2, &s->lc3, &s->mu1, &s->mu2, &s->mu3,
                      &s->gc1x, &s->gc1y, &s->gc2x, &s->gc2y, &s->gc3x, &s->gc3y, &s->grx,
                      &s->gry, &s->lmu1, &s->lmu2, &s->fsx, &s->fsy, &s->gbx, &s->gby,
                      &s->ux, &s->uy, &s->fax, &s->fay, &s->p, &s->d1x, &s->d1y, &s->d2x,
                      &s->d2y};
    for (size_t i = 0; i < sizeof all / sizeof all[0]; ++i) *all[i] = alloc_field(n);
    for (int k = 0; k < 9; ++k) {
        s->f1[k] = alloc_field(n); s->f2[k] = alloc_field(n); s->g[k] = alloc_field(n);
        s->fe1[k] = alloc_field(n); s->fe2[k] = alloc_field(n); s->ge[k] = alloc_field(n);
        s->F1[k] = alloc_field(n); s->F2[k] = alloc_field(n); s->Gk[k] = alloc_field(n);
        s->fp1[k] = alloc_field(n); s->fp2[k] = alloc_field(n); s->gp[k] = alloc_field(n);
    }
    *out = s;
    return 0;
}

/* ----------------------------------------------------------------- stencils */
/* Eq. 20b on c_i with the wetting ghosts of Eq. 42 across solid links (S2+S3).
 * comp = 0,1,2 selects c1, c2, c3. */
static void lap_c_wetting(orc_sim* s, int comp, const double* ci, double* lap) {
    const int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            if (s->mat[i]) { lap[i] = 0.0; continue; }
            double acc = 0.0;
            for (int k = 1; k < 9; ++k) {
                long j = nbr(s, x, y, k);
                double chat;
                if (s->cls[j] == 2) {
                    chat = ci[s->inner[j]];          /* Eq. 53: chi(x_u) = chi(x_f) */
                } else if (s->cls[j] == 1) {
                    const mat_t* m = &s->mats[s->mat[j] - 1];
                    double gh[3];
                    orc_wetting_ghost(s->fl.D, m->cos12, m->cos13, m->cos23,
                                      s->c1[i], s->c2[i], gh);
                    chat = gh[comp];
                } else {
                    chat = ci[j];
                }
                acc += 2.0 * W[k] * (chat - ci[i]) / CS2;
            }
            lap[i] = acc;
        }
}

/* value of chi seen across the link to neighbour j of fluid node i: a wall
 * neighbour takes chi(i) (symmetric ghost, Eq. 43), a velocity boundary
 * neighbour the value at the fluid node inside it (Eq. 53) */
static double across(const orc_sim* s, const double* chi, long i, long j) {
    if (s->cls[j] == 1) return chi[i];
    if (s->cls[j] == 2) return chi[s->inner[j]];
    return chi[j];
}

/* Eq. 20a with the symmetric ghost of Eq. 43 (solid neighbour takes chi(x_f)) */
int orc_grad_field(orc_sim* s, const double* chi, double* gx, double* gy) {
    const int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            if (s->mat[i]) { gx[i] = 0.0; gy[i] = 0.0; continue; }
            double ax = 0.0, ay = 0.0;
            for (int k = 1; k < 9; ++k) {
                long j = nbr(s, x, y, k);
                double v = across(s, chi, i, j);
                ax += W[k] * EX[k] * v / CS2;
                ay += W[k] * EY[k] * v / CS2;
            }
            gx[i] = ax;
            gy[i] = ay;
        }
    return 0;
}

/* Eq. 20b with the symmetric ghost of Eq. 43 */
int orc_lap_field(orc_sim* s, const double* chi, double* lap) {
    const int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            if (s->mat[i]) { lap[i] = 0.0; continue; }
            double acc = 0.0;
            for (int k = 1; k < 9; ++k) {
                long j = nbr(s, x, y, k);
                double v = across(s, chi, i, j);
                acc += 2.0 * W[k] * (v - chi[i]) / CS2;
            }
            lap[i] = acc;
        }
    return 0;
}

/* ------------------------------------------------------------------- steps */
/* S1: moments at fluid nodes */
static void s1_moments(orc_sim* s) {
    const orc_fluid* fl = &s->fl;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) {
            s->c1[i] = s->c2[i] = s->c3[i] = s->rho[i] = s->nu[i] = s->taug[i] = 0.0;
            continue;
        }
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 9; ++k) {
            a += s->f1[k][i];
            b += s->f2[k][i];
        }
        s->c1[i] = a;                         /* Eq. 13a */
        s->c2[i] = b;
        s->c3[i] = 1.0 - a - b;               /* Eq. 3 */
        s->rho[i] = a * fl->rho[0] + b * fl->rho[1] + s->c3[i] * fl->rho[2]; /* Eq. 14 */
        s->nu[i] = a * fl->nu[0] + b * fl->nu[1] + s->c3[i] * fl->nu[2];     /* Eq. 15 */
        s->taug[i] = s->nu[i] / CS2 + 0.5;    /* Eq. 18b */
    }
}

/* S2-S4: chemical potentials */
static void s4_mu(orc_sim* s) {
    lap_c_wetting(s, 0, s->c1, s->lc1);
    lap_c_wetting(s, 1, s->c2, s->lc2);
    lap_c_wetting(s, 2, s->c3, s->lc3);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) { s->mu1[i] = s->mu2[i] = s->mu3[i] = 0.0; continue; }
        double mu[3];
        orc_chem_potential(&s->fl, s->c1[i], s->c2[i], s->lc1[i], s->lc2[i], s->lc3[i], mu);
        s->mu1[i] = mu[0];
        s->mu2[i] = mu[1];
        s->mu3[i] = mu[2];
    }
}

/* S5-S10 */
static void s5_to_s10(orc_sim* s) {
    const orc_fluid* fl = &s->fl;
    /* S5 */
    orc_grad_field(s, s->c1, s->gc1x, s->gc1y);
    orc_grad_field(s, s->c2, s->gc2x, s->gc2y);
    orc_grad_field(s, s->c3, s->gc3x, s->gc3y);
    orc_grad_field(s, s->rho, s->grx, s->gry);
    orc_lap_field(s, s->mu1, s->lmu1);
    orc_lap_field(s, s->mu2, s->lmu2);
    /* S6 */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) {
            s->fsx[i] = s->fsy[i] = s->gbx[i] = s->gby[i] = s->ux[i] = s->uy[i] = 0.0;
            continue;
        }
        s->fsx[i] = s->mu1[i] * s->gc1x[i] + s->mu2[i] * s->gc2x[i] + s->mu3[i] * s->gc3x[i];
        s->fsy[i] = s->mu1[i] * s->gc1y[i] + s->mu2[i] * s->gc2y[i] + s->mu3[i] * s->gc3y[i];
        s->gbx[i] = s->rho[i] * fl->gravity[0];
        s->gby[i] = s->rho[i] * fl->gravity[1];
        double mx = 0.0, my = 0.0;
        for (int k = 0; k < 9; ++k) {
            mx += EX[k] * s->g[k][i];
            my += EY[k] * s->g[k][i];
        }
        s->ux[i] = (mx + 0.5 * (s->fsx[i] + s->gbx[i])) / s->rho[i]; /* Eq. 13b */
        s->uy[i] = (my + 0.5 * (s->fsy[i] + s->gby[i])) / s->rho[i];
    }
    /* S7, S8, S9 */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) {
            s->fax[i] = s->fay[i] = s->p[i] = 0.0;
            s->d1x[i] = s->d1y[i] = s->d2x[i] = s->d2y[i] = 0.0;
            continue;
        }
        double a = (fl->rho[0] - fl->rho[2]) * s->d.M[0] * s->lmu1[i]
                 + (fl->rho[1] - fl->rho[2]) * s->d.M[1] * s->lmu2[i];
        s->fax[i] = s->ux[i] * a;                                   /* Eq. 12 */
        s->fay[i] = s->uy[i] * a;
        double sum = 0.0;
        for (int k = 1; k < 9; ++k) sum += s->g[k][i];
        double udr = s->ux[i] * s->grx[i] + s->uy[i] * s->gry[i];
        s->p[i] = CS2 / (1.0 - W[0]) * (sum + 0.5 * udr + s->rho[i] * s_k(0, s->ux[i], s->uy[i])); /* Eq. 13c */
        /* Eq. 19 applied to chi = c_i u inside Eq. 11a */
        s->d1x[i] = s->c1[i] * s->ux[i] - s->c1o[i] * s->uxo[i];
        s->d1y[i] = s->c1[i] * s->uy[i] - s->c1o[i] * s->uyo[i];
        s->d2x[i] = s->c2[i] * s->ux[i] - s->c2o[i] * s->uxo[i];
        s->d2y[i] = s->c2[i] * s->uy[i] - s->c2o[i] * s->uyo[i];
    }
    /* S10 */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        double fe1[9], fe2[9], ge[9], F1[9], F2[9], G[9];
        if (s->mat[i]) {
            for (int k = 0; k < 9; ++k) {
                s->fe1[k][i] = s->fe2[k][i] = s->ge[k][i] = 0.0;
                s->F1[k][i] = s->F2[k][i] = s->Gk[k][i] = 0.0;
            }
            continue;
        }
        orc_equilibria(s->c1[i], s->c2[i], s->d.eta[0], s->d.eta[1], s->mu1[i], s->mu2[i],
                       s->rho[i], s->p[i], s->ux[i], s->uy[i], fe1, fe2, ge);
        orc_sources(fl->tau1, fl->tau2, s->taug[i], s->d1x[i], s->d1y[i], s->d2x[i],
                    s->d2y[i], s->ux[i], s->uy[i], s->grx[i], s->gry[i],
                    s->fsx[i] + s->gbx[i], s->fsy[i] + s->gby[i], s->fax[i], s->fay[i],
                    F1, F2, G);
        for (int k = 0; k < 9; ++k) {
            s->fe1[k][i] = fe1[k];
            s->fe2[k][i] = fe2[k];
            s->ge[k][i] = ge[k];
            s->F1[k][i] = F1[k];
            s->F2[k][i] = F2[k];
            s->Gk[k][i] = G[k];
        }
    }
}

int orc_eval(orc_sim* s) {
    if (!s->inited) { set_err("orc_eval before orc_init"); return -3; }
    s1_moments(s);
    s4_mu(s);
    s5_to_s10(s);
    return 0;
}

int orc_init(orc_sim* s, const double* c1, const double* c2,
             const double* ux, const double* uy) {
    const orc_fluid* fl = &s->fl;
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) {
            s->c1[i] = s->c2[i] = s->c3[i] = s->rho[i] = 0.0;
            continue;
        }
        s->c1[i] = c1[i];
        s->c2[i] = c2[i];
        s->c3[i] = 1.0 - c1[i] - c2[i];
        s->rho[i] = s->c1[i] * fl->rho[0] + s->c2[i] * fl->rho[1] + s->c3[i] * fl->rho[2];
    }
    s4_mu(s); /* mu from the initial c (S2-S4) */
    for (long i = 0; i < s->n; ++i) {
        double u0x = ux ? ux[i] : 0.0, u0y = uy ? uy[i] : 0.0;
        double fe1[9], fe2[9], ge[9];
        if (s->mat[i]) {
            for (int k = 0; k < 9; ++k) s->f1[k][i] = s->f2[k][i] = s->g[k][i] = 0.0;
            s->c1o[i] = s->c2o[i] = s->uxo[i] = s->uyo[i] = 0.0;
            continue;
        }
        orc_equilibria(s->c1[i], s->c2[i], s->d.eta[0], s->d.eta[1], s->mu1[i], s->mu2[i],
                       s->rho[i], 0.0, u0x, u0y, fe1, fe2, ge);
        for (int k = 0; k < 9; ++k) {
            s->f1[k][i] = fe1[k];
            s->f2[k][i] = fe2[k];
            s->g[k][i] = ge[k];
        }
        s->c1o[i] = s->c1[i];
        s->c2o[i] = s->c2[i];
        s->uxo[i] = u0x;
        s->uyo[i] = u0y;
    }
    s->inited = 1;
    return 0;
}

int orc_step(orc_sim* s, int nsteps) {
    if (!s->inited) { set_err("orc_step before orc_init"); return -3; }
    const int nx = s->nx, ny = s->ny;
    const double t1 = s->fl.tau1, t2 = s->fl.tau2;
    for (int it = 0; it < nsteps; ++it) {
        orc_eval(s); /* S1-S10 */
        /* S11: BGK collision, Eq. 45 */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < s->n; ++i) {
            if (s->mat[i]) continue;
            for (int k = 0; k < 9; ++k) {
                s->fp1[k][i] = s->f1[k][i] - (s->f1[k][i] - s->fe1[k][i]) / t1 + s->F1[k][i];
                s->fp2[k][i] = s->f2[k][i] - (s->f2[k][i] - s->fe2[k][i]) / t2 + s->F2[k][i];
                s->gp[k][i] = s->g[k][i] - (s->g[k][i] - s->ge[k][i]) / s->taug[i] + s->Gk[k][i];
            }
        }
        /* S11b: velocity boundary nodes (Eqs. 51-53).  The populations of x_u
         * are its equilibrium plus the non-equilibrium part of x_f (Eq. 51,
         * 52); the equilibrium uses x_f's c_i, mu_i, p, rho and the prescribed
         * u (Eq. 53).  x_u then collides like any node (Eq. 45), with source
         * terms (Eq. 11) formed the same way: every macroscopic quantity but u
         * from x_f, u = u_w (so d(c_i u)/dt = u_w (c_i - c_i^old) at x_f and
         * F_a = u_w times x_f's interfacial coefficient). */
#pragma omp parallel for schedule(static)
        for (long j = 0; j < s->n; ++j) {
            if (s->cls[j] != 2) continue;
            const long i = s->inner[j];
            const mat_t* m = &s->mats[s->mat[j] - 1];
            const double uwx = m->uw[0], uwy = m->uw[1];
            double fe1[9], fe2[9], ge[9], F1[9], F2[9], G[9];
            orc_equilibria(s->c1[i], s->c2[i], s->d.eta[0], s->d.eta[1], s->mu1[i], s->mu2[i],
                           s->rho[i], s->p[i], uwx, uwy, fe1, fe2, ge);
            const double dc1 = s->c1[i] - s->c1o[i], dc2 = s->c2[i] - s->c2o[i];
            const double a = (s->fl.rho[0] - s->fl.rho[2]) * s->d.M[0] * s->lmu1[i]
                           + (s->fl.rho[1] - s->fl.rho[2]) * s->d.M[1] * s->lmu2[i];
            orc_sources(t1, t2, s->taug[i], uwx * dc1, uwy * dc1, uwx * dc2, uwy * dc2,
                        uwx, uwy, s->grx[i], s->gry[i],
                        s->fsx[i] + s->gbx[i], s->fsy[i] + s->gby[i], uwx * a, uwy * a,
                        F1, F2, G);
            for (int k = 0; k < 9; ++k) {
                const double f1u = fe1[k] + (s->f1[k][i] - s->fe1[k][i]);   /* Eq. 51 */
                const double f2u = fe2[k] + (s->f2[k][i] - s->fe2[k][i]);
                const double gu = ge[k] + (s->g[k][i] - s->ge[k][i]);
                s->fp1[k][j] = f1u - (f1u - fe1[k]) / t1 + F1[k];           /* Eq. 45 */
                s->fp2[k][j] = f2u - (f2u - fe2[k]) / t2 + F2[k];
                s->gp[k][j] = gu - (gu - ge[k]) / s->taug[i] + G[k];
            }
        }
        /* S9 (history) now that the old values are consumed */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < s->n; ++i) {
            if (s->mat[i]) continue;
            s->c1o[i] = s->c1[i];
            s->c2o[i] = s->c2[i];
            s->uxo[i] = s->ux[i];
            s->uyo[i] = s->uy[i];
        }
        /* S12: pull streaming from fluid and velocity boundary nodes; a link
         * whose upstream node is a wall takes the node's own post-collision
         * population of the opposite direction (Eq. 44), plus the moving-wall
         * momentum term 2 w_k a e_k.u_w / c_s^2 with a = c_i for f^i and
         * a = rho for g. */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = (long)y * nx + x;
                if (s->mat[i]) continue;
                for (int k = 0; k < 9; ++k) {
                    long j = nbr(s, x, y, OPP[k]); /* x - e_k */
                    if (s->cls[j] != 1) {
                        s->f1[k][i] = s->fp1[k][j];
                        s->f2[k][i] = s->fp2[k][j];
                        s->g[k][i] = s->gp[k][j];
                    } else {
                        const mat_t* m = &s->mats[s->mat[j] - 1];
                        double eu = EX[k] * m->uw[0] + EY[k] * m->uw[1];
                        double b = 2.0 * W[k] * eu / CS2;
                        s->f1[k][i] = s->fp1[OPP[k]][i] + b * s->c1[i];
                        s->f2[k][i] = s->fp2[OPP[k]][i] + b * s->c2[i];
                        s->g[k][i] = s->gp[OPP[k]][i] + b * s->rho[i];
                    }
                }
            }
    }
    return 0;
}

int orc_fields(orc_sim* s, double* out) {
    int rc = orc_eval(s);
    if (rc) return rc;
    long n = s->n;
    double* src[ORC_NFIELDS] = {s->c1, s->c2, s->c3, s->rho, s->ux, s->uy, s->p,
                                s->mu1, s->mu2, s->mu3};
    for (int f = 0; f < ORC_NFIELDS; ++f)
        for (long i = 0; i < n; ++i) out[f * n + i] = s->mat[i] ? 0.0 : src[f][i];
    return 0;
}

int orc_stage(orc_sim* s, int id, double* out) {
    double* src[ORC_NSTAGE] = {s->lc1, s->lc2, s->lc3, s->gc1x, s->gc1y, s->gc2x, s->gc2y,
                               s->gc3x, s->gc3y, s->grx, s->gry, s->lmu1, s->lmu2,
                               s->fsx, s->fsy, s->fax, s->fay, s->taug, s->nu,
                               s->d1x, s->d1y, s->d2x, s->d2y};
    if (id < 0 || id >= ORC_NSTAGE) return -1;
    memcpy(out, src[id], (size_t)s->n * sizeof(double));
    return 0;
}

int orc_populations(orc_sim* s, double* out) {
    long n = s->n;
    for (int k = 0; k < 9; ++k) {
        memcpy(out + (long)k * n, s->f1[k], (size_t)n * sizeof(double));
        memcpy(out + (long)(9 + k) * n, s->f2[k], (size_t)n * sizeof(double));
        memcpy(out + (long)(18 + k) * n, s->g[k], (size_t)n * sizeof(double));
    }
    return 0;
}

int orc_set_populations(orc_sim* s, const double* in) {
    long n = s->n;
    for (int k = 0; k < 9; ++k) {
        memcpy(s->f1[k], in + (long)k * n, (size_t)n * sizeof(double));
        memcpy(s->f2[k], in + (long)(9 + k) * n, (size_t)n * sizeof(double));
        memcpy(s->g[k], in + (long)(18 + k) * n, (size_t)n * sizeof(double));
    }
    return 0;
}

int orc_history(orc_sim* s, double* out) {
    long n = s->n;
    memcpy(out, s->c1o, (size_t)n * sizeof(double));
    memcpy(out + n, s->c2o, (size_t)n * sizeof(double));
    memcpy(out + 2 * n, s->uxo, (size_t)n * sizeof(double));
    memcpy(out + 3 * n, s->uyo, (size_t)n * sizeof(double));
    return 0;
}

int orc_mass(orc_sim* s, double out[3]) {
    double m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) continue;
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 9; ++k) {
            a += s->f1[k][i];
            b += s->f2[k][i];
        }
        m1 += a;
        m2 += b;
        m3 += 1.0 - a - b;
    }
    out[0] = m1;
    out[1] = m2;
    out[2] = m3;
    return 0;
}
