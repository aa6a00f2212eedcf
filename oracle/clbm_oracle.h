/*
 * clbm_oracle.h -- FP64 CPU oracle of the double-distribution cascaded lattice
 * Boltzmann method of Fei & Luo, "Cascaded lattice Boltzmann method for
 * incompressible thermal flows with heat sources and general thermal boundary
 * conditions" (arXiv:1801.04577).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it. It shares no code, header, table or constant with
 * the GPU path.
 *
 * State convention: the oracle holds the PRE-collision populations f_i(x,t),
 * g_i(x,t) (after streaming). One call of oracle_step advances t -> t+1 by
 * collision (Eq. 7 and Eq. 23) followed by push streaming (Eq. 11, Eq. 21)
 * with half-way bounce-back for f and the general bounce-back scheme for g
 * (Eq. 26-28) at wall links.
 *
 * Storage is array-of-structures in host memory: f[(y*nx + x)*9 + i] and
 * g[(y*nx + x)*5 + i]; fields are row-major [ny][nx] (x fastest).
 */
#ifndef CLBM_ORACLE_H
#define CLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Side order: 0 = x-, 1 = x+, 2 = y-, 3 = y+. */
enum { ORACLE_PERIODIC = 0, ORACLE_WALL = 1 };

enum {
    ORACLE_OK = 0,
    ORACLE_ERR_INVALID_ARG = -1,
    ORACLE_ERR_UNSTABLE = -2,
    ORACLE_ERR_NOMEM = -3
};

typedef struct {
    int nx, ny;
    double nu;        /* kinematic viscosity, nu = (1/s_nu - 1/2)/3 (Sec. 2.1) */
    double alpha;     /* thermal diffusivity, alpha = (1/lambda_1 - 1/2) c_T^2 (Sec. 2.2) */
    double s_b;       /* bulk rate; NaN -> 1 */
    double s_4;       /* rate of k22; NaN -> 1 */
    double s_3;       /* rate of k21, k12; NaN -> no-slip rule (Sec. 3) */
    double lambda_0;  /* rate of thermal k00; NaN -> 1 */
    double lambda_2;  /* rate of thermal k20, k02; NaN -> Cui et al. rule (Sec. 3.1) */
    double g_beta;    /* Boussinesq coefficient, F_y = g_beta (T - T0) (Eq. 2) */
    double T0;        /* Boussinesq reference temperature (Eq. 2) */
    double Fx, Fy;    /* external body force F_v (Eq. 2) */
    double Q;         /* uniform heat source (Eq. 24) */
    int viscous_heating; /* add the viscous dissipation nu * Phi to Q (Sec. 3.2); needs g_beta = 0 */
    int kind[4];      /* ORACLE_PERIODIC or ORACLE_WALL per side */
    double u_wall[4]; /* tangential speed of a moving wall (x- and x+: along y; y-, y+: along x) */
    double b1[4], b2[4], b3[4]; /* thermal wall data: b1 dT/dn + b2 T = b3, n outward */
    const double* Q_field; /* NULL, or a heat source per node [ny][nx] added to Q (Sec. 3.2,
                              a spatially variable source); read by the lattice calls, not
                              by oracle_collide; the caller keeps it alive */
} oracle_params;

typedef struct oracle_sim oracle_sim;

int oracle_version(void);

/* Relaxation rates actually used: out = {s_nu, s_b, s_3, s_4, lambda_0, lambda_1, lambda_2}. */
int oracle_rates(const oracle_params* p, double out[7]);

/* Dense matrices as printed (row-major). */
void oracle_matrix_M(double out[81]);                       /* Eq. (6a) */
void oracle_matrix_N(double ux, double uy, double out[81]); /* Eq. (6b) */
void oracle_matrix_MT(double out[25]);                      /* Eq. (16) */
void oracle_matrix_NT(double ux, double uy, double out[25]); /* Eq. (17) */
void oracle_matrix_Minv(double out[81]);  /* numerical inverse of Eq. (6a) */
void oracle_matrix_MTinv(double out[25]); /* numerical inverse of Eq. (16) */

/* Discrete equilibria from the central-moment equilibria Eq. (9) and Eq. (19). */
void oracle_equilibrium(double rho, double ux, double uy, double T, double f[9], double g[5]);

/* One collision at one node. macro_out = {rho, ux, uy, T} (pre-collision, Eq. 12, 25). */
int oracle_collide(const oracle_params* p, const double f[9], const double g[5],
                   double f_post[9], double g_post[5], double macro_out[4]);

int  oracle_create(const oracle_params* p, oracle_sim** out);
void oracle_destroy(oracle_sim* s);
/* Equilibrium initial state from fields [ny][nx]; any NULL field -> rho=1, u=0, T=T0. */
int  oracle_init(oracle_sim* s, const double* rho, const double* ux, const double* uy,
                 const double* T);
int  oracle_step(oracle_sim* s, long nsteps, int nthreads);
long oracle_step_count(const oracle_sim* s);
/* Macroscopic fields at the current time (pre-collision); NULL outputs are skipped. */
int  oracle_macros(const oracle_sim* s, double* rho, double* ux, double* uy, double* T);
int  oracle_get_state(const oracle_sim* s, double* f, double* g);
int  oracle_set_state(oracle_sim* s, const double* f, const double* g, long step);
/* Post-collision populations of the current state (does not advance time). */
int  oracle_post_collision(const oracle_sim* s, double* f_post, double* g_post, int nthreads);
/* Per wall node of side `side`: wall temperature (Eq. 28) and outward normal
 * derivative (Eq. 27) at the current time. Length ny for x-sides, nx for y-sides. */
int  oracle_wall_values(const oracle_sim* s, int side, double* Tw, double* dTdn);

#ifdef __cplusplus
}
#endif
#endif
