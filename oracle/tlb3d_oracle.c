/*
 * tlb3d_oracle.c -- plain FP64 CPU oracle of the three-dimensional version
 * of the ternary phase-field lattice Boltzmann step with the ternary wetting
 * boundary scheme (Liang et al., arXiv:1710.09534; the paper states its
 * model on D2Q9 "without loss of generality", Sec. II.A).  TEST
 * INFRASTRUCTURE ONLY, like tlb_oracle.c: loaded by the tests and the
 * benchmark's CPU-baseline leg, never by the GPU library.
 *
 * The lattice is D3Q19 (rest, six axis links, twelve edge diagonals; weights
 * 1/3, 1/18, 1/36; c_s^2 = 1/3), which carries the isotropic gradient and
 * Laplacian of Eq. 20.  Every equation is the one of the D2Q9 model with
 * sums over the 19 links and 3-vectors: moments (Eqs. 3, 13a, 14, 15, 18b),
 * wetting ghosts (Eq. 42), chemical potentials (Eq. 8, plus the lambda > 0
 * part of Eq. 6), symmetric ghosts (Eq. 43), forces and velocity (Eq. 13b),
 * interfacial force (Eq. 12), pressure (Eq. 13c with w_0 = 1/3), Euler time
 * derivative (Eq. 19), equilibria (Eqs. 2, 4), sources (Eq. 11), BGK
 * collision (Eq. 45), pull streaming with half-way bounce-back (Eq. 44) and
 * the moving-wall term.  One array per intermediate, in the paper's order
 * (S6-S10 of a node share one loop).  Built with -O2 -ffp-contract=off;
 * OpenMP splits z-planes only, so results do not depend on the thread count.
 * Walls only: the velocity boundary of Sec. III.D is not part of the 3-D
 * version.
 */
#include "tlb_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19: k = 0 rest; 1-6 axis links (+x, -x, +y, -y, +z, -z); 7-18 edge
 * diagonals in pairs (e, -e). */
static const int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double CS2 = 1.0 / 3.0;

static int opp3(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }
static double w3(int k) { return k == 0 ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

static char g_err3[512];
static void set_err3(const char* m) { snprintf(g_err3, sizeof g_err3, "%s", m); }
const char* orc3_last_error(void) { return g_err3; }

void orc3_lattice(int ex[19], int ey[19], int ez[19], double w[19], int opp[19]) {
    for (int k = 0; k < 19; ++k) {
        ex[k] = EX[k];
        ey[k] = EY[k];
        ez[k] = EZ[k];
        w[k] = w3(k);
        opp[k] = opp3(k);
    }
}

typedef struct {
    double cos12, cos13, cos23;
    double uw[3];
} mat3_t;

struct orc3_sim {
    int nx, ny, nz, px, py, pz;
    long n;
    orc_fluid fl;
    double gz;
    orc_derived d;
    uint8_t* mat;
    mat3_t* mats;
    int nmat, inited;
    double *f1[19], *f2[19], *g[19];
    double *c1o, *c2o, *uxo, *uyo, *uzo;
    double *c1, *c2, *c3, *rho, *taug;
    double *lc1, *lc2, *lc3, *mu1, *mu2, *mu3;
    double *gc1[3], *gc2[3], *gc3[3], *gr[3], *lmu1, *lmu2;
    double *fs[3], *gb[3], *u[3], *fa[3], *p, *d1[3], *d2[3];
    double *fe1[19], *fe2[19], *ge[19], *F1[19], *F2[19], *Gk[19];
    double *fp1[19], *fp2[19], *gp[19];
};

static long nbr3(const orc3_sim* s, int x, int y, int z, int dx, int dy, int dz) {
    int xn = x + dx, yn = y + dy, zn = z + dz;
    if (xn < 0 || xn >= s->nx) {
        if (!s->px) return -1;
        xn = (xn + s->nx) % s->nx;
    }
    if (yn < 0 || yn >= s->ny) {
        if (!s->py) return -1;
        yn = (yn + s->ny) % s->ny;
    }
    if (zn < 0 || zn >= s->nz) {
        if (!s->pz) return -1;
        zn = (zn + s->nz) % s->nz;
    }
    return ((long)zn * s->ny + yn) * s->nx + xn;
}

#define ALL_FIELDS(X)                                                                          \
    X(c1o) X(c2o) X(uxo) X(uyo) X(uzo) X(c1) X(c2) X(c3) X(rho) X(taug) X(lc1) X(lc2) X(lc3)   \
    X(mu1) X(mu2) X(mu3) X(lmu1) X(lmu2) X(p)

void orc3_destroy(orc3_sim* s) {
    if (!s) return;
#define FREE1(a) free(s->a);
    ALL_FIELDS(FREE1)
#undef FREE1
    for (int a = 0; a < 3; ++a) {
        free(s->gc1[a]); free(s->gc2[a]); free(s->gc3[a]); free(s->gr[a]);
        free(s->fs[a]); free(s->gb[a]); free(s->u[a]); free(s->fa[a]);
        free(s->d1[a]); free(s->d2[a]);
    }
    for (int k = 0; k < 19; ++k) {
        free(s->f1[k]); free(s->f2[k]); free(s->g[k]);
        free(s->fe1[k]); free(s->fe2[k]); free(s->ge[k]);
        free(s->F1[k]); free(s->F2[k]); free(s->Gk[k]);
        free(s->fp1[k]); free(s->fp2[k]); free(s->gp[k]);
    }
    free(s->mat);
    free(s->mats);
    free(s);
}

int orc3_create(int nx, int ny, int nz, const orc_fluid* fl, double gravity_z, int px, int py,
                int pz, const uint8_t* material, const orc_material* mats, int n_mats,
                orc3_sim** out) {
    *out = NULL;
    if (nx < 3 || ny < 3 || nz < 3 || !fl || !material || n_mats < 0 || (n_mats > 0 && !mats)) {
        set_err3("invalid sizes or null pointer");
        return -1;
    }
    orc_derived d;
    if (fl->D <= 0 || fl->M0 <= 0 || fl->tau1 <= 0.5 || fl->tau2 <= 0.5) {
        set_err3("D, M0 must be > 0 and tau_i > 1/2");
        return -2;
    }
    if (orc_params(fl, &d) != 0) {
        set_err3("inadmissible surface tensions or lambda");
        return -2;
    }
    orc3_sim* s = (orc3_sim*)calloc(1, sizeof(orc3_sim));
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->px = px != 0; s->py = py != 0; s->pz = pz != 0;
    s->n = (long)nx * ny * nz;
    s->fl = *fl;
    s->gz = gravity_z;
    s->d = d;
    s->nmat = n_mats;
    s->mats = (mat3_t*)calloc((size_t)(n_mats > 0 ? n_mats : 1), sizeof(mat3_t));
    const double d2r = acos(-1.0) / 180.0;
    for (int m = 0; m < n_mats; ++m) {
        double c12;
        if (mats[m].kind != ORC_WALL) {
            set_err3("only wall materials in 3-D");
            orc3_destroy(s);
            return -1;
        }
        if (orc_cos12(fl, mats[m].theta13_deg, mats[m].theta23_deg, &c12) != 0) {
            set_err3("contact angles give |cos theta12| > 1 (Eq. 39)");
            orc3_destroy(s);
            return -2;
        }
        s->mats[m].cos12 = c12;
        s->mats[m].cos13 = cos(mats[m].theta13_deg * d2r);
        s->mats[m].cos23 = cos(mats[m].theta23_deg * d2r);
        s->mats[m].uw[0] = mats[m].wall_u[0];
        s->mats[m].uw[1] = mats[m].wall_u[1];
        s->mats[m].uw[2] = 0.0;
    }
    s->mat = (uint8_t*)malloc((size_t)s->n);
    memcpy(s->mat, material, (size_t)s->n);
    for (long i = 0; i < s->n; ++i)
        if (s->mat[i] > n_mats) {
            set_err3("material id exceeds the material table");
            orc3_destroy(s);
            return -1;
        }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (s->mat[((long)z * ny + y) * nx + x]) continue;
                for (int k = 1; k < 19; ++k)
                    if (nbr3(s, x, y, z, EX[k], EY[k], EZ[k]) < 0) {
                        set_err3("fluid node on the edge of a non-periodic direction");
                        orc3_destroy(s);
                        return -1;
                    }
            }
    long n = s->n;
#define ALLOC1(a) s->a = (double*)calloc((size_t)n, sizeof(double));
    ALL_FIELDS(ALLOC1)
#undef ALLOC1
    for (int a = 0; a < 3; ++a) {
        s->gc1[a] = (double*)calloc((size_t)n, sizeof(double));
        s->gc2[a] = (double*)calloc((size_t)n, sizeof(double));
        s->gc3[a] = (double*)calloc((size_t)n, sizeof(double));
        s->gr[a] = (double*)calloc((size_t)n, sizeof(double));
        s->fs[a] = (double*)calloc((size_t)n, sizeof(double));
        s->gb[a] = (double*)calloc((size_t)n, sizeof(double));
        s->u[a] = (double*)calloc((size_t)n, sizeof(double));
        s->fa[a] = (double*)calloc((size_t)n, sizeof(double));
        s->d1[a] = (double*)calloc((size_t)n, sizeof(double));
        s->d2[a] = (double*)calloc((size_t)n, sizeof(double));
    }
    for (int k = 0; k < 19; ++k) {
        s->f1[k] = (double*)calloc((size_t)n, sizeof(double));
        s->f2[k] = (double*)calloc((size_t)n, sizeof(double));
        s->g[k] = (double*)calloc((size_t)n, sizeof(double));
        s->fe1[k] = (double*)calloc((size_t)n, sizeof(double));
        s->fe2[k] = (double*)calloc((size_t)n, sizeof(double));
        s->ge[k] = (double*)calloc((size_t)n, sizeof(double));
        s->F1[k] = (double*)calloc((size_t)n, sizeof(double));
        s->F2[k] = (double*)calloc((size_t)n, sizeof(double));
        s->Gk[k] = (double*)calloc((size_t)n, sizeof(double));
        s->fp1[k] = (double*)calloc((size_t)n, sizeof(double));
        s->fp2[k] = (double*)calloc((size_t)n, sizeof(double));
        s->gp[k] = (double*)calloc((size_t)n, sizeof(double));
    }
    *out = s;
    return 0;
}

/* s_k(u) of Eq. 4 on D3Q19 */
static double sk3(int k, const double u[3]) {
    double eu = EX[k] * u[0] + EY[k] * u[1] + EZ[k] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return w3(k) * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* node index helpers */
#define IDX(x, y, z) (((long)(z) * s->ny + (y)) * s->nx + (x))

/* S2 + S3: Laplacian of c_i (Eq. 20b) with the wetting ghosts of Eq. 42 */
static void lap_c_wetting3(orc3_sim* s, int comp, const double* ci, double* lap) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long i = IDX(x, y, z);
                if (s->mat[i]) { lap[i] = 0.0; continue; }
                double acc = 0.0;
                for (int k = 1; k < 19; ++k) {
                    long j = nbr3(s, x, y, z, EX[k], EY[k], EZ[k]);
                    double chat;
                    if (s->mat[j]) {
                        const mat3_t* m = &s->mats[s->mat[j] - 1];
                        double gh[3];
                        orc_wetting_ghost(s->fl.D, m->cos12, m->cos13, m->cos23, s->c1[i],
                                          s->c2[i], gh);
                        chat = gh[comp];
                    } else {
                        chat = ci[j];
                    }
                    acc += 2.0 * w3(k) * (chat - ci[i]) / CS2;
                }
                lap[i] = acc;
            }
}

/* Eq. 20a with the symmetric ghost of Eq. 43 */
int orc3_grad_field(orc3_sim* s, const double* chi, double* gx, double* gy, double* gz) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long i = IDX(x, y, z);
                if (s->mat[i]) { gx[i] = gy[i] = gz[i] = 0.0; continue; }
                double a = 0.0, b = 0.0, c = 0.0;
                for (int k = 1; k < 19; ++k) {
                    long j = nbr3(s, x, y, z, EX[k], EY[k], EZ[k]);
                    double v = s->mat[j] ? chi[i] : chi[j];
                    a += w3(k) * EX[k] * v / CS2;
                    b += w3(k) * EY[k] * v / CS2;
                    c += w3(k) * EZ[k] * v / CS2;
                }
                gx[i] = a; gy[i] = b; gz[i] = c;
            }
    return 0;
}

/* Eq. 20b with the symmetric ghost of Eq. 43 */
int orc3_lap_field(orc3_sim* s, const double* chi, double* lap) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long i = IDX(x, y, z);
                if (s->mat[i]) { lap[i] = 0.0; continue; }
                double acc = 0.0;
                for (int k = 1; k < 19; ++k) {
                    long j = nbr3(s, x, y, z, EX[k], EY[k], EZ[k]);
                    double v = s->mat[j] ? chi[i] : chi[j];
                    acc += 2.0 * w3(k) * (v - chi[i]) / CS2;
                }
                lap[i] = acc;
            }
    return 0;
}

/* S1 */
static void s1_moments3(orc3_sim* s) {
    const orc_fluid* fl = &s->fl;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) { s->c1[i] = s->c2[i] = s->c3[i] = s->rho[i] = s->taug[i] = 0.0; continue; }
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 19; ++k) { a += s->f1[k][i]; b += s->f2[k][i]; }
        s->c1[i] = a;
        s->c2[i] = b;
        s->c3[i] = 1.0 - a - b;
        s->rho[i] = a * fl->rho[0] + b * fl->rho[1] + s->c3[i] * fl->rho[2];
        double nu = a * fl->nu[0] + b * fl->nu[1] + s->c3[i] * fl->nu[2];
        s->taug[i] = nu / CS2 + 0.5;
    }
}

/* S2-S4 */
static void s4_mu3(orc3_sim* s) {
    lap_c_wetting3(s, 0, s->c1, s->lc1);
    lap_c_wetting3(s, 1, s->c2, s->lc2);
    lap_c_wetting3(s, 2, s->c3, s->lc3);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) { s->mu1[i] = s->mu2[i] = s->mu3[i] = 0.0; continue; }
        double mu[3];
        orc_chem_potential(&s->fl, s->c1[i], s->c2[i], s->lc1[i], s->lc2[i], s->lc3[i], mu);
        s->mu1[i] = mu[0]; s->mu2[i] = mu[1]; s->mu3[i] = mu[2];
    }
}

/* S5-S10 */
static void s5_to_s10_3(orc3_sim* s) {
    const orc_fluid* fl = &s->fl;
    const double grav[3] = {fl->gravity[0], fl->gravity[1], s->gz};
    orc3_grad_field(s, s->c1, s->gc1[0], s->gc1[1], s->gc1[2]);
    orc3_grad_field(s, s->c2, s->gc2[0], s->gc2[1], s->gc2[2]);
    orc3_grad_field(s, s->c3, s->gc3[0], s->gc3[1], s->gc3[2]);
    orc3_grad_field(s, s->rho, s->gr[0], s->gr[1], s->gr[2]);
    orc3_lap_field(s, s->mu1, s->lmu1);
    orc3_lap_field(s, s->mu2, s->lmu2);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) {
            for (int a = 0; a < 3; ++a)
                s->fs[a][i] = s->gb[a][i] = s->u[a][i] = s->fa[a][i] = s->d1[a][i] = s->d2[a][i] = 0.0;
            s->p[i] = 0.0;
            for (int k = 0; k < 19; ++k)
                s->fe1[k][i] = s->fe2[k][i] = s->ge[k][i] = s->F1[k][i] = s->F2[k][i] = s->Gk[k][i] = 0.0;
            continue;
        }
        double m[3] = {0.0, 0.0, 0.0}, u[3], F[3];
        for (int k = 0; k < 19; ++k) {
            m[0] += EX[k] * s->g[k][i];
            m[1] += EY[k] * s->g[k][i];
            m[2] += EZ[k] * s->g[k][i];
        }
        /* S6: F_s (potential form), G = rho g, u (Eq. 13b) */
        for (int a = 0; a < 3; ++a) {
            s->fs[a][i] = s->mu1[i] * s->gc1[a][i] + s->mu2[i] * s->gc2[a][i] + s->mu3[i] * s->gc3[a][i];
            s->gb[a][i] = s->rho[i] * grav[a];
            F[a] = s->fs[a][i] + s->gb[a][i];
            u[a] = (m[a] + 0.5 * F[a]) / s->rho[i];
            s->u[a][i] = u[a];
        }
        /* S7: F_a (Eq. 12) */
        double am = (fl->rho[0] - fl->rho[2]) * s->d.M[0] * s->lmu1[i]
                  + (fl->rho[1] - fl->rho[2]) * s->d.M[1] * s->lmu2[i];
        for (int a = 0; a < 3; ++a) s->fa[a][i] = u[a] * am;
        /* S8: p (Eq. 13c) */
        double sum = 0.0, udr = 0.0;
        for (int k = 1; k < 19; ++k) sum += s->g[k][i];
        for (int a = 0; a < 3; ++a) udr += u[a] * s->gr[a][i];
        s->p[i] = CS2 / (1.0 - w3(0)) * (sum + 0.5 * udr + s->rho[i] * sk3(0, u));
        /* S9: d(c_i u)/dt (Eq. 19) */
        const double uo[3] = {s->uxo[i], s->uyo[i], s->uzo[i]};
        for (int a = 0; a < 3; ++a) {
            s->d1[a][i] = s->c1[i] * u[a] - s->c1o[i] * uo[a];
            s->d2[a][i] = s->c2[i] * u[a] - s->c2o[i] * uo[a];
        }
        /* S10: equilibria (Eqs. 2, 4) and sources (Eq. 11, F_a outside the factor) */
        const double e1 = s->d.eta[0] * s->mu1[i], e2 = s->d.eta[1] * s->mu2[i];
        const double fsg = 1.0 - 1.0 / (2.0 * s->taug[i]);
        for (int k = 0; k < 19; ++k) {
            const double w = w3(k);
            const double eu = EX[k] * u[0] + EY[k] * u[1] + EZ[k] * u[2];
            const double sk = sk3(k, u);
            if (k == 0) {
                s->fe1[k][i] = s->c1[i] + (w - 1.0) * e1;
                s->fe2[k][i] = s->c2[i] + (w - 1.0) * e2;
                s->ge[k][i] = s->p[i] / CS2 * (w - 1.0) + s->rho[i] * sk;
            } else {
                s->fe1[k][i] = w * e1 + w * s->c1[i] * eu / CS2;
                s->fe2[k][i] = w * e2 + w * s->c2[i] * eu / CS2;
                s->ge[k][i] = s->p[i] / CS2 * w + s->rho[i] * sk;
            }
            double ed1 = EX[k] * s->d1[0][i] + EY[k] * s->d1[1][i] + EZ[k] * s->d1[2][i];
            double ed2 = EX[k] * s->d2[0][i] + EY[k] * s->d2[1][i] + EZ[k] * s->d2[2][i];
            s->F1[k][i] = (1.0 - 1.0 / (2.0 * fl->tau1)) * w * ed1 / CS2;
            s->F2[k][i] = (1.0 - 1.0 / (2.0 * fl->tau2)) * w * ed2 / CS2;
            const double ek[3] = {(double)EX[k], (double)EY[k], (double)EZ[k]};
            double acc = 0.0, efa = 0.0;
            for (int a = 0; a < 3; ++a) {
                acc += (ek[a] - u[a]) * (sk * s->gr[a][i] + (sk + w) * F[a] / CS2);
                efa += ek[a] * s->fa[a][i];
            }
            s->Gk[k][i] = fsg * acc + w * efa / CS2;
        }
    }
}

int orc3_eval(orc3_sim* s) {
    if (!s->inited) { set_err3("orc3_eval before orc3_init"); return -3; }
    s1_moments3(s);
    s4_mu3(s);
    s5_to_s10_3(s);
    return 0;
}

int orc3_init(orc3_sim* s, const double* c1, const double* c2, const double* ux,
              const double* uy, const double* uz) {
    const orc_fluid* fl = &s->fl;
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) { s->c1[i] = s->c2[i] = s->c3[i] = s->rho[i] = 0.0; continue; }
        s->c1[i] = c1[i];
        s->c2[i] = c2[i];
        s->c3[i] = 1.0 - c1[i] - c2[i];
        s->rho[i] = c1[i] * fl->rho[0] + c2[i] * fl->rho[1] + s->c3[i] * fl->rho[2];
    }
    s4_mu3(s);
    for (long i = 0; i < s->n; ++i) {
        const double u[3] = {ux ? ux[i] : 0.0, uy ? uy[i] : 0.0, uz ? uz[i] : 0.0};
        if (s->mat[i]) {
            for (int k = 0; k < 19; ++k) s->f1[k][i] = s->f2[k][i] = s->g[k][i] = 0.0;
            s->c1o[i] = s->c2o[i] = s->uxo[i] = s->uyo[i] = s->uzo[i] = 0.0;
            continue;
        }
        const double e1 = s->d.eta[0] * s->mu1[i], e2 = s->d.eta[1] * s->mu2[i];
        for (int k = 0; k < 19; ++k) {
            const double w = w3(k);
            const double eu = EX[k] * u[0] + EY[k] * u[1] + EZ[k] * u[2];
            if (k == 0) {
                s->f1[k][i] = s->c1[i] + (w - 1.0) * e1;
                s->f2[k][i] = s->c2[i] + (w - 1.0) * e2;
            } else {
                s->f1[k][i] = w * e1 + w * s->c1[i] * eu / CS2;
                s->f2[k][i] = w * e2 + w * s->c2[i] * eu / CS2;
            }
            s->g[k][i] = s->rho[i] * sk3(k, u);   /* p = 0 */
        }
        s->c1o[i] = s->c1[i];
        s->c2o[i] = s->c2[i];
        s->uxo[i] = u[0];
        s->uyo[i] = u[1];
        s->uzo[i] = u[2];
    }
    s->inited = 1;
    return 0;
}

int orc3_step(orc3_sim* s, int nsteps) {
    if (!s->inited) { set_err3("orc3_step before orc3_init"); return -3; }
    const double t1 = s->fl.tau1, t2 = s->fl.tau2;
    for (int it = 0; it < nsteps; ++it) {
        orc3_eval(s);
        /* S11: BGK collision (Eq. 45) */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < s->n; ++i) {
            if (s->mat[i]) continue;
            for (int k = 0; k < 19; ++k) {
                s->fp1[k][i] = s->f1[k][i] - (s->f1[k][i] - s->fe1[k][i]) / t1 + s->F1[k][i];
                s->fp2[k][i] = s->f2[k][i] - (s->f2[k][i] - s->fe2[k][i]) / t2 + s->F2[k][i];
                s->gp[k][i] = s->g[k][i] - (s->g[k][i] - s->ge[k][i]) / s->taug[i] + s->Gk[k][i];
            }
        }
        /* S9 history */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < s->n; ++i) {
            if (s->mat[i]) continue;
            s->c1o[i] = s->c1[i];
            s->c2o[i] = s->c2[i];
            s->uxo[i] = s->u[0][i];
            s->uyo[i] = s->u[1][i];
            s->uzo[i] = s->u[2][i];
        }
        /* S12: pull streaming, half-way bounce-back (Eq. 44) with the
         * moving-wall term 2 w_k a e_k.u_w / c_s^2 (a = c_i, rho) */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y)
                for (int x = 0; x < s->nx; ++x) {
                    long i = IDX(x, y, z);
                    if (s->mat[i]) continue;
                    for (int k = 0; k < 19; ++k) {
                        long j = nbr3(s, x, y, z, -EX[k], -EY[k], -EZ[k]);
                        if (!s->mat[j]) {
                            s->f1[k][i] = s->fp1[k][j];
                            s->f2[k][i] = s->fp2[k][j];
                            s->g[k][i] = s->gp[k][j];
                        } else {
                            const mat3_t* m = &s->mats[s->mat[j] - 1];
                            double eu = EX[k] * m->uw[0] + EY[k] * m->uw[1] + EZ[k] * m->uw[2];
                            double b = 2.0 * w3(k) * eu / CS2;
                            const int o = opp3(k);
                            s->f1[k][i] = s->fp1[o][i] + b * s->c1[i];
                            s->f2[k][i] = s->fp2[o][i] + b * s->c2[i];
                            s->g[k][i] = s->gp[o][i] + b * s->rho[i];
                        }
                    }
                }
    }
    return 0;
}

/* fields: c1, c2, c3, rho, ux, uy, uz, p, mu1, mu2, mu3 (11 x n); boundary nodes 0 */
int orc3_fields(orc3_sim* s, double* out) {
    int rc = orc3_eval(s);
    if (rc) return rc;
    double* src[11] = {s->c1, s->c2, s->c3, s->rho, s->u[0], s->u[1], s->u[2], s->p,
                       s->mu1, s->mu2, s->mu3};
    for (int f = 0; f < 11; ++f)
        for (long i = 0; i < s->n; ++i) out[f * s->n + i] = s->mat[i] ? 0.0 : src[f][i];
    return 0;
}

/* populations f1[0..18], f2[0..18], g[0..18] (57 x n) */
int orc3_populations(orc3_sim* s, double* out) {
    for (int k = 0; k < 19; ++k) {
        memcpy(out + (long)k * s->n, s->f1[k], (size_t)s->n * sizeof(double));
        memcpy(out + (long)(19 + k) * s->n, s->f2[k], (size_t)s->n * sizeof(double));
        memcpy(out + (long)(38 + k) * s->n, s->g[k], (size_t)s->n * sizeof(double));
    }
    return 0;
}

int orc3_mass(orc3_sim* s, double out[3]) {
    double m1 = 0.0, m2 = 0.0, m3 = 0.0;
    for (long i = 0; i < s->n; ++i) {
        if (s->mat[i]) continue;
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 19; ++k) { a += s->f1[k][i]; b += s->f2[k][i]; }
        m1 += a;
        m2 += b;
        m3 += 1.0 - a - b;
    }
    out[0] = m1; out[1] = m2; out[2] = m3;
    return 0;
}
