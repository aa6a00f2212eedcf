/*
 * clbm_oracle.c -- FP64 CPU oracle of the cascaded LBM for incompressible
 * thermal flows (Fei & Luo, arXiv:1801.04577).
 *
 * TEST INFRASTRUCTURE. Plain, slow and literal on purpose: the matrices are
 * the dense ones printed in the paper, the inverses are taken numerically,
 * every node is collided with dense matrix-vector products and the result is
 * pushed to its neighbours. Nothing here is blocked, fused or reordered beyond
 * what the paper's equations state. No code is shared with the GPU library.
 *
 * One time step, in the paper's order:
 *   Sec. 2.3 Eq. (25)  T = sum g + Q/2
 *   Sec. 2   Eq. (2)   F = -g beta (T - T0) + F_v, gravity along -y
 *   Sec. 2.1 Eq. (12)  rho = sum f, rho u = sum f e + F/2
 *   Sec. 2.1 Eq. (6)-(10) cascaded collision with consistent forcing
 *   Sec. 2.1           f* = M^-1 N^-1 Gamma~*
 *   Sec. 2.2 Eq. (15)-(19), Sec. 2.3 Eq. (23)-(24) thermal collision with source
 *   Sec. 2.2 Eq. (20)  g* = M_T^-1 N_T^-1 Gamma~T*
 *   Eq. (11), Eq. (21) streaming; Sec. 3 half-way bounce-back for f;
 *   Sec. 2.3 Eq. (26)-(28) general bounce-back for g.
 *
 * Parity status of each function is recorded in the test suite that pins it.
 */
#include "clbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q9 9
#define Q5 5

/* Eq. (3): D2Q9 velocities; the D2Q5 set is the first five. */
static const int EX[Q9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* c_s^2 = 1/3 (Sec. 2.1, after Eq. 9); c_T^2 = 2/5 (Sec. 3). */
static const double CS2 = 1.0 / 3.0;
static const double CT2 = 2.0 / 5.0;

/* Eq. (6a), as printed. Rows: k00 k10 k01 k20 k02 k11 k21 k12 k22 (Eq. 5). */
static const double M_PRINTED[Q9][Q9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 1, 0, 1, 0, 1, 1, 1, 1},
    {0, 0, 1, 0, 1, 1, 1, 1, 1},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 1, 1, 1, 1},
};

/* Eq. (16), as printed. Rows: k00 k10 k01 k20 k02 (Eq. 14). */
static const double MT_PRINTED[Q5][Q5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {0, 1, 0, 1, 0},
    {0, 0, 1, 0, 1},
};

int oracle_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Dense linear algebra                                                      */
/* ------------------------------------------------------------------------ */

/* Gauss-Jordan elimination with partial pivoting: inv = A^-1 (n x n, row-major). */
static int invert_dense(int n, const double* A, double* inv)
{
    double a[Q9 * Q9 * 2];
    int w = 2 * n;
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) {
            a[r * w + c] = A[r * n + c];
            a[r * w + n + c] = (r == c) ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r * w + col]) > fabs(a[piv * w + col])) piv = r;
        if (a[piv * w + col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < w; ++c) {
                double t = a[col * w + c];
                a[col * w + c] = a[piv * w + c];
                a[piv * w + c] = t;
            }
        double d = a[col * w + col];
        for (int c = 0; c < w; ++c) a[col * w + c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double m = a[r * w + col];
            if (m == 0.0) continue;
            for (int c = 0; c < w; ++c) a[r * w + c] -= m * a[col * w + c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) inv[r * n + c] = a[r * w + n + c];
    return 0;
}

static void matvec(int n, const double* A, const double* x, double* y)
{
    for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += A[r * n + c] * x[c];
        y[r] = s;
    }
}

/* Solve L x = b for lower-triangular L (forward substitution): applies L^-1. */
static void solve_lower(int n, const double* L, const double* b, double* x)
{
    for (int r = 0; r < n; ++r) {
        double s = b[r];
        for (int c = 0; c < r; ++c) s -= L[r * n + c] * x[c];
        x[r] = s / L[r * n + r];
    }
}

/* ------------------------------------------------------------------------ */
/* Matrices of the paper                                                     */
/* ------------------------------------------------------------------------ */

void oracle_matrix_M(double out[81])
{
    for (int r = 0; r < Q9; ++r)
        for (int c = 0; c < Q9; ++c) out[r * Q9 + c] = M_PRINTED[r][c];
}

void oracle_matrix_MT(double out[25])
{
    for (int r = 0; r < Q5; ++r)
        for (int c = 0; c < Q5; ++c) out[r * Q5 + c] = MT_PRINTED[r][c];
}

/* Eq. (6b), entry by entry as printed. */
void oracle_matrix_N(double ux, double uy, double out[81])
{
    double N[Q9][Q9];
    memset(N, 0, sizeof N);
    double ux2 = ux * ux, uy2 = uy * uy;
    N[0][0] = 1;
    N[1][0] = -ux;            N[1][1] = 1;
    N[2][0] = -uy;            N[2][2] = 1;
    N[3][0] = ux2;            N[3][1] = -2 * ux;  N[3][3] = 1;
    N[4][0] = uy2;            N[4][2] = -2 * uy;  N[4][4] = 1;
    N[5][0] = ux * uy;        N[5][1] = -uy;      N[5][2] = -ux;   N[5][5] = 1;
    N[6][0] = -ux2 * uy;      N[6][1] = 2 * ux * uy; N[6][2] = ux2; N[6][3] = -uy;
    N[6][5] = -2 * ux;        N[6][6] = 1;
    N[7][0] = -uy2 * ux;      N[7][1] = uy2;      N[7][2] = 2 * ux * uy; N[7][4] = -ux;
    N[7][5] = -2 * uy;        N[7][7] = 1;
    N[8][0] = ux2 * uy2;      N[8][1] = -2 * ux * uy2; N[8][2] = -2 * uy * ux2;
    N[8][3] = uy2;            N[8][4] = ux2;      N[8][5] = 4 * ux * uy;
    N[8][6] = -2 * uy;        N[8][7] = -2 * ux;  N[8][8] = 1;
    for (int r = 0; r < Q9; ++r)
        for (int c = 0; c < Q9; ++c) out[r * Q9 + c] = N[r][c];
}

/* Eq. (17), as printed. */
void oracle_matrix_NT(double ux, double uy, double out[25])
{
    double N[Q5][Q5];
    memset(N, 0, sizeof N);
    N[0][0] = 1;
    N[1][0] = -ux;      N[1][1] = 1;
    N[2][0] = -uy;      N[2][2] = 1;
    N[3][0] = ux * ux;  N[3][1] = -2 * ux; N[3][3] = 1;
    N[4][0] = uy * uy;  N[4][2] = -2 * uy; N[4][4] = 1;
    for (int r = 0; r < Q5; ++r)
        for (int c = 0; c < Q5; ++c) out[r * Q5 + c] = N[r][c];
}

void oracle_matrix_Minv(double out[81])
{
    double M[81];
    oracle_matrix_M(M);
    invert_dense(Q9, M, out);
}

void oracle_matrix_MTinv(double out[25])
{
    double M[25];
    oracle_matrix_MT(M);
    invert_dense(Q5, M, out);
}

/* ------------------------------------------------------------------------ */
/* Relaxation rates                                                          */
/* ------------------------------------------------------------------------ */

int oracle_rates(const oracle_params* p, double out[7])
{
    if (!(p->nu > 0.0) || !(p->alpha > 0.0)) return ORACLE_ERR_INVALID_ARG;
    /* Sec. 2.1: nu = (1/s_nu - 1/2)/3. */
    double s_nu = 1.0 / (3.0 * p->nu + 0.5);
    double s_b = isnan(p->s_b) ? 1.0 : p->s_b;
    double s_4 = isnan(p->s_4) ? 1.0 : p->s_4;
    /* Sec. 3: no-slip rule s_3 = (16 - 8 s_nu)/(8 - s_nu). */
    double s_3 = isnan(p->s_3) ? (16.0 - 8.0 * s_nu) / (8.0 - s_nu) : p->s_3;
    double l0 = isnan(p->lambda_0) ? 1.0 : p->lambda_0;
    /* Sec. 2.2: alpha = (1/lambda_1 - 1/2) c_T^2. */
    double l1 = 1.0 / (p->alpha / CT2 + 0.5);
    /* Sec. 3.1: lambda_2 = 12 (lambda_1 - 2)/(lambda_1 - 12). */
    double l2 = isnan(p->lambda_2) ? 12.0 * (l1 - 2.0) / (l1 - 12.0) : p->lambda_2;
    out[0] = s_nu; out[1] = s_b; out[2] = s_3; out[3] = s_4;
    out[4] = l0;   out[5] = l1;  out[6] = l2;
    for (int k = 0; k < 7; ++k)
        if (!(out[k] > 0.0 && out[k] < 2.0)) return ORACLE_ERR_UNSTABLE;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Equilibria and the collision of one node                                  */
/* ------------------------------------------------------------------------ */

/* Eq. (9) and Eq. (19) mapped back to populations: f = M^-1 N^-1 Gamma~eq. */
static void equilibrium_with(const double* Minv, const double* MTinv, double rho, double ux,
                             double uy, double T, double f[9], double g[5])
{
    double N[81], NT[25];
    oracle_matrix_N(ux, uy, N);
    oracle_matrix_NT(ux, uy, NT);
    double keq[Q9] = {rho, 0, 0, rho * CS2, rho * CS2, 0, 0, 0, rho * CS2 * CS2};
    double kteq[Q5] = {T, 0, 0, T * CT2, T * CT2};
    double raw[Q9], rawt[Q5];
    solve_lower(Q9, N, keq, raw);
    matvec(Q9, Minv, raw, f);
    solve_lower(Q5, NT, kteq, rawt);
    matvec(Q5, MTinv, rawt, g);
}

void oracle_equilibrium(double rho, double ux, double uy, double T, double f[9], double g[5])
{
    double Minv[81], MTinv[25];
    oracle_matrix_Minv(Minv);
    oracle_matrix_MTinv(MTinv);
    equilibrium_with(Minv, MTinv, rho, ux, uy, T, f, g);
}

typedef struct {
    double s_nu, s_b, s_3, s_4, l0, l1, l2;
    double S[Q9 * Q9];
    double ST[Q5 * Q5];
    double Minv[Q9 * Q9];
    double MTinv[Q5 * Q5];
    double M[Q9 * Q9];
    double MT[Q5 * Q5];
} collide_ctx;

static int make_ctx(const oracle_params* p, collide_ctx* c)
{
    double r[7];
    int st = oracle_rates(p, r);
    if (st != ORACLE_OK) return st;
    c->s_nu = r[0]; c->s_b = r[1]; c->s_3 = r[2]; c->s_4 = r[3];
    c->l0 = r[4];   c->l1 = r[5];  c->l2 = r[6];
    /* Eq. (8): S = diag([0,0,0], [[s+, s-],[s-, s+]], [s_nu, s_3, s_3, s_4]). */
    double sp = 0.5 * (c->s_b + c->s_nu), sm = 0.5 * (c->s_b - c->s_nu);
    memset(c->S, 0, sizeof c->S);
    c->S[3 * Q9 + 3] = sp; c->S[3 * Q9 + 4] = sm;
    c->S[4 * Q9 + 3] = sm; c->S[4 * Q9 + 4] = sp;
    c->S[5 * Q9 + 5] = c->s_nu;
    c->S[6 * Q9 + 6] = c->s_3;
    c->S[7 * Q9 + 7] = c->s_3;
    c->S[8 * Q9 + 8] = c->s_4;
    /* Sec. 2.2: S_T = diag(lambda_0, lambda_1, lambda_1, lambda_2, lambda_2). */
    memset(c->ST, 0, sizeof c->ST);
    c->ST[0] = c->l0;
    c->ST[1 * Q5 + 1] = c->l1; c->ST[2 * Q5 + 2] = c->l1;
    c->ST[3 * Q5 + 3] = c->l2; c->ST[4 * Q5 + 4] = c->l2;
    oracle_matrix_M(c->M);
    oracle_matrix_MT(c->MT);
    if (invert_dense(Q9, c->M, c->Minv) != 0) return ORACLE_ERR_INVALID_ARG;
    if (invert_dense(Q5, c->MT, c->MTinv) != 0) return ORACLE_ERR_INVALID_ARG;
    return ORACLE_OK;
}

/* Viscous dissipation of Sec. 3.2 (Q = nu (du/dy)^2 in a channel), in general
 * nu [(d_x u_y + d_y u_x)^2 + (d_x u_x - d_y u_y)^2] for divergence-free flow. The
 * strain rates come from the pre-collision central moments: to first order in the
 * Chapman-Enskog expansion k11 = -(rho c_s^2/s_nu)(d_x u_y + d_y u_x) and
 * k20 - k02 = -(2 rho c_s^2/s_nu)(d_x u_x - d_y u_y). */
static double dissipation(const oracle_params* p, const collide_ctx* c, const double* cen, double rho)
{
    double shear = -c->s_nu * cen[5] / (CS2 * rho);
    double normal = -c->s_nu * (cen[3] - cen[4]) / (2.0 * CS2 * rho);
    return p->nu * (shear * shear + normal * normal);
}

/* Heat source at node k: the uniform Q, plus the caller's source field at k when there is
 * one (k < 0: none), plus, with viscous heating, the dissipation evaluated from the
 * pre-collision populations f (velocity from Eq. 12 with F = F_v). */
static double local_source(const oracle_params* p, const collide_ctx* c, const double* f, long k)
{
    const double Q = p->Q + ((p->Q_field && k >= 0) ? p->Q_field[k] : 0.0);
    if (!p->viscous_heating) return Q;
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q9; ++i) {
        rho += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    double ux = (jx + 0.5 * p->Fx) / rho, uy = (jy + 0.5 * p->Fy) / rho;
    double N[Q9 * Q9], raw[Q9], cen[Q9];
    oracle_matrix_N(ux, uy, N);
    matvec(Q9, c->M, f, raw);
    matvec(Q9, N, raw, cen);
    return Q + dissipation(p, c, cen, rho);
}

static void collide_node(const oracle_params* p, const collide_ctx* c, long k, const double* f,
                         const double* g, double* fp, double* gp, double* macro)
{
    /* Eq. (25): temperature with the source correction. */
    const double Qn = local_source(p, c, f, k);
    double T = 0.0;
    for (int i = 0; i < Q5; ++i) T += g[i];
    T += 0.5 * Qn;
    /* Eq. (2): Boussinesq force, gravity along -y so -g beta (T-T0) points along +y. */
    double Fx = p->Fx;
    double Fy = p->Fy + p->g_beta * (T - p->T0);
    /* Eq. (12). */
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q9; ++i) {
        rho += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    double ux = (jx + 0.5 * Fx) / rho;
    double uy = (jy + 0.5 * Fy) / rho;

    /* Flow: Eq. (6)-(10), then f* = M^-1 N^-1 Gamma~*. */
    double N[Q9 * Q9];
    oracle_matrix_N(ux, uy, N);
    double raw[Q9], cen[Q9];
    matvec(Q9, c->M, f, raw);
    matvec(Q9, N, raw, cen);
    double keq[Q9] = {rho, 0, 0, rho * CS2, rho * CS2, 0, 0, 0, rho * CS2 * CS2};
    double C[Q9] = {0, Fx, Fy, 0, 0, 0, CS2 * Fy, CS2 * Fx, 0};
    double post[Q9];
    for (int r = 0; r < Q9; ++r) {
        double s = 0.0;
        for (int k = 0; k < Q9; ++k) {
            double Srk = c->S[r * Q9 + k];
            double I = (r == k) ? 1.0 : 0.0;
            s += (I - Srk) * cen[k] + Srk * keq[k] + (I - 0.5 * Srk) * C[k];
        }
        post[r] = s;
    }
    double rawp[Q9];
    solve_lower(Q9, N, post, rawp);
    matvec(Q9, c->Minv, rawp, fp);

    /* Temperature: Eq. (15)-(19) with the source of Eq. (23)-(24), then Eq. (20). */
    double NT[Q5 * Q5];
    oracle_matrix_NT(ux, uy, NT);
    double rt[Q5], ct[Q5];
    matvec(Q5, c->MT, g, rt);
    matvec(Q5, NT, rt, ct);
    double kteq[Q5] = {T, 0, 0, T * CT2, T * CT2};
    double R[Q5] = {Qn, 0, 0, Qn * CT2, Qn * CT2};
    double pt[Q5];
    for (int r = 0; r < Q5; ++r) {
        double s = 0.0;
        for (int k = 0; k < Q5; ++k) {
            double Srk = c->ST[r * Q5 + k];
            double I = (r == k) ? 1.0 : 0.0;
            s += (I - Srk) * ct[k] + Srk * kteq[k] + (I - 0.5 * Srk) * R[k];
        }
        pt[r] = s;
    }
    double rawt[Q5];
    solve_lower(Q5, NT, pt, rawt);
    matvec(Q5, c->MTinv, rawt, gp);

    if (macro) {
        macro[0] = rho; macro[1] = ux; macro[2] = uy; macro[3] = T;
    }
}

int oracle_collide(const oracle_params* p, const double f[9], const double g[5],
                   double f_post[9], double g_post[5], double macro_out[4])
{
    collide_ctx c;
    int st = make_ctx(p, &c);
    if (st != ORACLE_OK) return st;
    collide_node(p, &c, -1, f, g, f_post, g_post, macro_out);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Lattice                                                                   */
/* ------------------------------------------------------------------------ */

struct oracle_sim {
    oracle_params p;
    collide_ctx c;
    double w[Q9];          /* rest equilibrium weights f_i^eq(1, 0) from Eq. (9) */
    double *f, *g;         /* pre-collision state at time t */
    double *fn, *gn;       /* streaming target */
    double *fp, *gp;       /* post-collision scratch */
    double *rho, *T;       /* pre-collision rho and T at time t */
    long step;
};

static int opposite(int i)
{
    for (int k = 0; k < Q9; ++k)
        if (EX[k] == -EX[i] && EY[k] == -EY[i]) return k;
    return -1;
}

int oracle_create(const oracle_params* p, oracle_sim** out)
{
    if (!p || !out) return ORACLE_ERR_INVALID_ARG;
    *out = NULL;
    if (p->nx < 1 || p->ny < 1) return ORACLE_ERR_INVALID_ARG;
    if (p->kind[0] != p->kind[1] || p->kind[2] != p->kind[3]) return ORACLE_ERR_INVALID_ARG;
    /* Eq. (27) needs a second fluid layer next to every wall. */
    if (p->kind[0] == ORACLE_WALL && p->nx < 2) return ORACLE_ERR_INVALID_ARG;
    if (p->kind[2] == ORACLE_WALL && p->ny < 2) return ORACLE_ERR_INVALID_ARG;
    for (int s = 0; s < 4; ++s) {
        if (p->kind[s] != ORACLE_PERIODIC && p->kind[s] != ORACLE_WALL)
            return ORACLE_ERR_INVALID_ARG;
        if (p->kind[s] == ORACLE_WALL && p->b1[s] == 0.0 && p->b2[s] == 0.0)
            return ORACLE_ERR_INVALID_ARG;
    }
    /* The dissipation source is computed from the velocity field, which must not depend on
     * the temperature it produces (no buoyancy). */
    if (p->viscous_heating && p->g_beta != 0.0) return ORACLE_ERR_INVALID_ARG;
    oracle_sim* s = (oracle_sim*)calloc(1, sizeof *s);
    if (!s) return ORACLE_ERR_NOMEM;
    s->p = *p;
    int st = make_ctx(p, &s->c);
    if (st != ORACLE_OK) {
        free(s);
        return st;
    }
    double g5[Q5];
    oracle_equilibrium(1.0, 0.0, 0.0, 0.0, s->w, g5);
    size_t n = (size_t)p->nx * (size_t)p->ny;
    s->f = (double*)calloc(n * Q9, sizeof(double));
    s->fn = (double*)calloc(n * Q9, sizeof(double));
    s->fp = (double*)calloc(n * Q9, sizeof(double));
    s->g = (double*)calloc(n * Q5, sizeof(double));
    s->gn = (double*)calloc(n * Q5, sizeof(double));
    s->gp = (double*)calloc(n * Q5, sizeof(double));
    s->rho = (double*)calloc(n, sizeof(double));
    s->T = (double*)calloc(n, sizeof(double));
    if (!s->f || !s->fn || !s->fp || !s->g || !s->gn || !s->gp || !s->rho || !s->T) {
        oracle_destroy(s);
        return ORACLE_ERR_NOMEM;
    }
    *out = s;
    return oracle_init(s, NULL, NULL, NULL, NULL);
}

void oracle_destroy(oracle_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fn); free(s->fp);
    free(s->g); free(s->gn); free(s->gp);
    free(s->rho); free(s->T);
    free(s);
}

int oracle_init(oracle_sim* s, const double* rho, const double* ux, const double* uy,
                const double* T)
{
    const long n = (long)s->p.nx * (long)s->p.ny;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long k = 0; k < n; ++k) {
        double r = rho ? rho[k] : 1.0;
        double vx = ux ? ux[k] : 0.0;
        double vy = uy ? uy[k] : 0.0;
        double t = T ? T[k] : s->p.T0;
        equilibrium_with(s->c.Minv, s->c.MTinv, r, vx, vy, t, s->f + k * Q9, s->g + k * Q5);
    }
    s->step = 0;
    return ORACLE_OK;
}

long oracle_step_count(const oracle_sim* s) { return s->step; }

/* Wall temperature from Eq. (28) with n . e_i = 1 and dx = 1 (n outward, e_i pointing
 * from the fluid node to the wall). T1, T2: first- and second-layer temperatures. */
static double wall_temperature(const oracle_params* p, int side, double T1, double T2)
{
    double b1 = p->b1[side], b2 = p->b2[side], b3 = p->b3[side];
    double ne = 1.0, dx = 1.0;
    return (9.0 * b1 * T1 - b1 * T2 + 3.0 * ne * dx * b3) / (8.0 * b1 + 3.0 * ne * dx * b2);
}

/* The side a link leaves through when it moves by (ex, ey) from (x, y), or -1 if the
 * target stays inside (periodic directions wrap). *tx, *ty receive the wrapped target. */
static int crossed_sides(const oracle_params* p, int x, int y, int ex, int ey, int* tx, int* ty,
                         int* xside, int* yside)
{
    int X = x + ex, Y = y + ey;
    *xside = -1;
    *yside = -1;
    if (X < 0 || X >= p->nx) {
        if (p->kind[0] == ORACLE_PERIODIC) X = (X + p->nx) % p->nx;
        else *xside = (X < 0) ? 0 : 1;
    }
    if (Y < 0 || Y >= p->ny) {
        if (p->kind[2] == ORACLE_PERIODIC) Y = (Y + p->ny) % p->ny;
        else *yside = (Y < 0) ? 2 : 3;
    }
    *tx = X;
    *ty = Y;
    return (*xside >= 0 || *yside >= 0);
}

static void collide_all(const oracle_sim* s, const double* f, const double* g, double* fp,
                        double* gp, double* rho, double* T, int nthreads)
{
    int nx = s->p.nx, ny = s->p.ny;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)y * nx + x;
            double m[4];
            collide_node(&s->p, &s->c, (long)k, f + k * Q9, g + k * Q5, fp + k * Q9, gp + k * Q5, m);
            if (rho) rho[k] = m[0];
            if (T) T[k] = m[3];
        }
    }
}

static void stream_all(oracle_sim* s, int nthreads)
{
    const oracle_params* p = &s->p;
    int nx = p->nx, ny = p->ny;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)y * nx + x;
            for (int i = 0; i < Q9; ++i) {
                int tx, ty, xs, ys;
                int hit = crossed_sides(p, x, y, EX[i], EY[i], &tx, &ty, &xs, &ys);
                int ib = opposite(i);
                if (!hit) {
                    /* Eq. (11) and Eq. (21). */
                    size_t kt = (size_t)ty * nx + tx;
                    s->fn[kt * Q9 + i] = s->fp[k * Q9 + i];
                    if (i < Q5) s->gn[kt * Q5 + i] = s->gp[k * Q5 + i];
                    continue;
                }
                /* Half-way bounce-back for f (Sec. 3); a moving wall adds the momentum
                 * exchange term -2 w_i rho (e_i . u_w)/c_s^2. */
                double uwx = (ys >= 0) ? p->u_wall[ys] : 0.0;
                double uwy = (xs >= 0) ? p->u_wall[xs] : 0.0;
                double eu = EX[i] * uwx + EY[i] * uwy;
                s->fn[k * Q9 + ib] = s->fp[k * Q9 + i] - 2.0 * s->w[i] * s->rho[k] * eu / CS2;
                if (i >= 1 && i < Q5) {
                    /* Eq. (26)-(28): general bounce-back. The wall is crossed along one
                     * axis; T1 at this node, T2 one node further from the wall. */
                    int side = (xs >= 0) ? xs : ys;
                    int x2 = x - EX[i], y2 = y - EY[i];
                    double T1 = s->T[k];
                    double T2 = s->T[(size_t)y2 * nx + x2];
                    double Tw = wall_temperature(p, side, T1, T2);
                    s->gn[k * Q5 + ib] = -s->gp[k * Q5 + i] + CT2 * Tw;
                }
            }
        }
    }
}

int oracle_step(oracle_sim* s, long nsteps, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    for (long n = 0; n < nsteps; ++n) {
        collide_all(s, s->f, s->g, s->fp, s->gp, s->rho, s->T, nthreads);
        stream_all(s, nthreads);
        double* t = s->f; s->f = s->fn; s->fn = t;
        t = s->g; s->g = s->gn; s->gn = t;
        s->step++;
    }
    return ORACLE_OK;
}

int oracle_macros(const oracle_sim* s, double* rho, double* ux, double* uy, double* T)
{
    const oracle_params* p = &s->p;
    size_t n = (size_t)p->nx * (size_t)p->ny;
    for (size_t k = 0; k < n; ++k) {
        const double* f = s->f + k * Q9;
        const double* g = s->g + k * Q5;
        double t = 0.0;
        for (int i = 0; i < Q5; ++i) t += g[i];
        t += 0.5 * local_source(p, &s->c, f, (long)k);     /* Eq. (25) */
        double Fx = p->Fx, Fy = p->Fy + p->g_beta * (t - p->T0); /* Eq. (2) */
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < Q9; ++i) {
            r += f[i];
            jx += f[i] * EX[i];
            jy += f[i] * EY[i];
        }
        if (rho) rho[k] = r;                               /* Eq. (12) */
        if (ux) ux[k] = (jx + 0.5 * Fx) / r;
        if (uy) uy[k] = (jy + 0.5 * Fy) / r;
        if (T) T[k] = t;
    }
    return ORACLE_OK;
}

int oracle_get_state(const oracle_sim* s, double* f, double* g)
{
    size_t n = (size_t)s->p.nx * (size_t)s->p.ny;
    if (f) memcpy(f, s->f, n * Q9 * sizeof(double));
    if (g) memcpy(g, s->g, n * Q5 * sizeof(double));
    return ORACLE_OK;
}

int oracle_set_state(oracle_sim* s, const double* f, const double* g, long step)
{
    size_t n = (size_t)s->p.nx * (size_t)s->p.ny;
    if (f) memcpy(s->f, f, n * Q9 * sizeof(double));
    if (g) memcpy(s->g, g, n * Q5 * sizeof(double));
    s->step = step;
    return ORACLE_OK;
}

int oracle_post_collision(const oracle_sim* s, double* f_post, double* g_post, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    size_t n = (size_t)s->p.nx * (size_t)s->p.ny;
    double* fp = (double*)malloc(n * Q9 * sizeof(double));
    double* gp = (double*)malloc(n * Q5 * sizeof(double));
    if (!fp || !gp) {
        free(fp);
        free(gp);
        return ORACLE_ERR_NOMEM;
    }
    collide_all(s, s->f, s->g, fp, gp, NULL, NULL, nthreads);
    if (f_post) memcpy(f_post, fp, n * Q9 * sizeof(double));
    if (g_post) memcpy(g_post, gp, n * Q5 * sizeof(double));
    free(fp);
    free(gp);
    return ORACLE_OK;
}

int oracle_wall_values(const oracle_sim* s, int side, double* Tw, double* dTdn)
{
    const oracle_params* p = &s->p;
    if (side < 0 || side > 3 || p->kind[side] != ORACLE_WALL) return ORACLE_ERR_INVALID_ARG;
    int nx = p->nx, ny = p->ny;
    double* T = (double*)malloc((size_t)nx * ny * sizeof(double));
    if (!T) return ORACLE_ERR_NOMEM;
    oracle_macros(s, NULL, NULL, NULL, T);
    int len = (side < 2) ? ny : nx;
    for (int j = 0; j < len; ++j) {
        int x1, y1, x2, y2;
        if (side == 0)      { x1 = 0;      y1 = j; x2 = 1;      y2 = j; }
        else if (side == 1) { x1 = nx - 1; y1 = j; x2 = nx - 2; y2 = j; }
        else if (side == 2) { x1 = j; y1 = 0;      x2 = j; y2 = 1; }
        else                { x1 = j; y1 = ny - 1; x2 = j; y2 = ny - 2; }
        double T1 = T[(size_t)y1 * nx + x1], T2 = T[(size_t)y2 * nx + x2];
        double tw = wall_temperature(p, side, T1, T2);
        if (Tw) Tw[j] = tw;
        /* Eq. (27) with n . e_i = 1, dx = 1. */
        if (dTdn) dTdn[j] = (8.0 * tw - 9.0 * T1 + T2) / 3.0;
    }
    free(T);
    return ORACLE_OK;
}
