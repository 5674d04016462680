/*
 * tlb_oracle.h -- slow, plain FP64 CPU oracle for the ternary phase-field
 * lattice Boltzmann step with the ternary wetting boundary scheme of
 * Liang, Xu, Chen, Chai & Shi, "Lattice Boltzmann modeling of wall-bounded
 * ternary fluid flows" (arXiv:1710.09534).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the GPU library and must never be
 * used as a fallback for it.
 *
 * Every step of the method is a separate full-field loop with its own
 * array, in the order of the paper's algorithm (Sec. II.A, Eqs. 1-20, and
 * Sec. II.B, Eqs. 40-45).  Parity of a function that no test pins to the
 * paper or to mathematics is marked "parity unpinned" in its comment.
 *
 * Conventions: lattice units (dx = dt = 1); fields are row-major with x
 * fastest, index = y*nx + x, y = 0 is the bottom row.  material[idx] == 0
 * is a fluid node, m >= 1 a boundary node of material mats[m-1]: a solid
 * wall, or a velocity boundary node (Sec. III, Eqs. 51-53).
 */
#ifndef TLB_ORACLE_H
#define TLB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double sigma12, sigma13, sigma23; /* Eq. 7 */
    double D;                         /* interface thickness, Eq. 8 */
    double M0;                        /* M_i = M0 / lambda_i, Eq. 12 */
    double tau1, tau2;                /* Eq. 1a */
    double rho[3], nu[3];             /* Eqs. 14-15 */
    double gravity[2];                /* body force G = rho * gravity */
    double lambda;                    /* coefficient of the c1^2 c2^2 c3^2 term of the
                                         bulk energy, Eq. 5 (>= 0; 0 gives Eq. 8) */
} orc_fluid;

/* material kinds */
enum { ORC_WALL = 0, ORC_VELOCITY = 1 };

typedef struct {
    double theta13_deg, theta23_deg;  /* theta12 follows from Eq. 39 (walls only) */
    double wall_u[2];                 /* wall velocity (ORC_WALL), or the prescribed
                                         boundary velocity (ORC_VELOCITY) */
    int kind;                         /* ORC_WALL: solid wall with the wetting scheme
                                         (Eqs. 42-44); ORC_VELOCITY: velocity boundary
                                         node of the non-equilibrium extrapolation
                                         scheme (Eqs. 51-53), allowed only in the
                                         bottom or top row of a lattice that is not
                                         periodic in y, with a fluid node directly
                                         inside it */
} orc_material;

/* derived parameters, see orc_params() */
typedef struct {
    double lambda[3], lambdaT;  /* Eqs. 7, 9 */
    double M[2];                /* Eq. 12 */
    double eta[2];              /* Eq. 18a solved for eta, one per component */
} orc_derived;

typedef struct orc_sim orc_sim;

/* field ids for orc_fields / orc_stage */
enum {
    ORC_C1 = 0, ORC_C2, ORC_C3, ORC_RHO, ORC_UX, ORC_UY, ORC_P,
    ORC_MU1, ORC_MU2, ORC_MU3, ORC_NFIELDS
};

/* intermediate arrays exposed for tests (valid after orc_eval) */
enum {
    ORC_S_LAPC1 = 0, ORC_S_LAPC2, ORC_S_LAPC3,
    ORC_S_GC1X, ORC_S_GC1Y, ORC_S_GC2X, ORC_S_GC2Y, ORC_S_GC3X, ORC_S_GC3Y,
    ORC_S_GRX, ORC_S_GRY, ORC_S_LAPMU1, ORC_S_LAPMU2,
    ORC_S_FSX, ORC_S_FSY, ORC_S_FAX, ORC_S_FAY, ORC_S_TAUG, ORC_S_NU,
    ORC_S_D1X, ORC_S_D1Y, ORC_S_D2X, ORC_S_D2Y,
    ORC_NSTAGE
};

/* ---- pure functions (pins) ---- */
void   orc_lattice(int ex[9], int ey[9], double w[9], int opp[9]);
int    orc_params(const orc_fluid* fl, orc_derived* out);
/* cos(theta12) from Eq. 39; returns 0 if |cos| <= 1, else -1 */
int    orc_cos12(const orc_fluid* fl, double theta13_deg, double theta23_deg, double* cos12);
/* ghost order parameters of Eq. 42 for one fluid node and one solid link */
void   orc_wetting_ghost(double D, double cos12, double cos13, double cos23,
                         double c1, double c2, double out[3]);
/* chemical potentials of Eq. 6 (Eq. 8 when lambda = 0) from c and the
 * Laplacians of c */
void   orc_chem_potential(const orc_fluid* fl, double c1, double c2,
                          double lap1, double lap2, double lap3, double mu[3]);
/* f^{i,eq} (Eq. 2a) and g^eq (Eq. 2b, Eq. 4) */
void   orc_equilibria(double c1, double c2, double eta1, double eta2,
                      double mu1, double mu2, double rho, double p,
                      double ux, double uy,
                      double feq1[9], double feq2[9], double geq[9]);
/* source terms of Eq. 11: F^1_k, F^2_k (from dt(c_i u) = D_i) and G_k */
void   orc_sources(double tau1, double tau2, double taug,
                   double d1x, double d1y, double d2x, double d2y,
                   double ux, double uy, double grx, double gry,
                   double fx, double fy, double fax, double fay,
                   double F1[9], double F2[9], double G[9]);

/* ---- whole-lattice simulation ---- */
/* returns 0 on success, <0 on invalid input (message via orc_last_error) */
int    orc_create(int nx, int ny, const orc_fluid* fl, int periodic_x, int periodic_y,
                  const uint8_t* material, const orc_material* mats, int n_mats,
                  orc_sim** out);
void   orc_destroy(orc_sim* s);
const char* orc_last_error(void);
/* equilibrium initialisation (p = 0, history = (c1, c2, u0)); ux/uy nullable */
int    orc_init(orc_sim* s, const double* c1, const double* c2,
                const double* ux, const double* uy);
/* evaluate S1-S10 on the current populations (no state change) */
int    orc_eval(orc_sim* s);
/* advance nsteps full steps */
int    orc_step(orc_sim* s, int nsteps);
/* macroscopic fields at the current time: ORC_NFIELDS x (ny*nx), field-major.
 * Solid nodes read as 0. */
int    orc_fields(orc_sim* s, double* out);
/* copy an intermediate array (after orc_eval or orc_step) */
int    orc_stage(orc_sim* s, int id, double* out);
/* current populations f(x,t): 27 x (ny*nx): f1[0..8], f2[0..8], g[0..8] */
int    orc_populations(orc_sim* s, double* out);
int    orc_set_populations(orc_sim* s, const double* in);
/* history (c1, c2, ux, uy at t-1): 4 x (ny*nx) */
int    orc_history(orc_sim* s, double* out);
/* sum of c1, c2, c3 over fluid nodes, sequential row-major order */
int    orc_mass(orc_sim* s, double out[3]);
/* gradient / Laplacian of an arbitrary field with the symmetric ghost rule of Eq. 43 */
int    orc_grad_field(orc_sim* s, const double* chi, double* gx, double* gy);
int    orc_lap_field(orc_sim* s, const double* chi, double* lap);
/* number of threads the oracle's loops use */
int    orc_num_threads(void);
void   orc_set_num_threads(int n);

/* ---- three-dimensional version (tlb3d_oracle.c): D3Q19, walls only ---- */
typedef struct orc3_sim orc3_sim;
void   orc3_lattice(int ex[19], int ey[19], int ez[19], double w[19], int opp[19]);
/* material: [nz][ny][nx], 0 fluid, m >= 1 wall material mats[m-1] (tangential
 * wall velocity (wall_u[0], wall_u[1], 0)); gravity = (fl->gravity[0],
 * fl->gravity[1], gravity_z) */
int    orc3_create(int nx, int ny, int nz, const orc_fluid* fl, double gravity_z,
                   int px, int py, int pz, const uint8_t* material,
                   const orc_material* mats, int n_mats, orc3_sim** out);
void   orc3_destroy(orc3_sim* s);
const char* orc3_last_error(void);
int    orc3_init(orc3_sim* s, const double* c1, const double* c2, const double* ux,
                 const double* uy, const double* uz);
int    orc3_eval(orc3_sim* s);
int    orc3_step(orc3_sim* s, int nsteps);
/* c1, c2, c3, rho, ux, uy, uz, p, mu1, mu2, mu3: 11 x n, boundary nodes 0 */
int    orc3_fields(orc3_sim* s, double* out);
/* f1[0..18], f2[0..18], g[0..18]: 57 x n */
int    orc3_populations(orc3_sim* s, double* out);
int    orc3_mass(orc3_sim* s, double out[3]);
int    orc3_grad_field(orc3_sim* s, const double* chi, double* gx, double* gy, double* gz);
int    orc3_lap_field(orc3_sim* s, const double* chi, double* lap);

#ifdef __cplusplus
}
#endif
#endif
