/*
 * FP64 CPU oracle for the 13-moment double-distribution lattice Boltzmann step
 * on D3Q39 (Latt, Coreixas, Beny, Parmigiani, "Efficient supersonic flows
 * through high-order guided equilibrium with lattice Boltzmann", 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * library never does.  It shares no source with the HIP path.
 *
 * Every routine follows the paper's statement of the method in the order the
 * paper gives it, with no blocking, fusion or reordering:
 *   - velocity set: Sec. 3, the E_{3,7}^{39} lattice (D3Q39);
 *   - Maxwell-Boltzmann target moments: Sec. 2, Eq. (eq:EqMomentsTensor),
 *     with the 13 constraints of Eq. (eq:13constraints);
 *   - exponential equilibrium: Sec. 2, Eq. (eq:discrete-equilibrium);
 *   - Newton-Raphson for the Lagrange multipliers: Sec. 3 and the algorithm
 *     table of Sec. 5 (warm start from the previous time step); a secant
 *     (limited-memory BFGS) variant that never evaluates the Jacobian, for
 *     the choice of root finder that Sec. 6 leaves open;
 *   - polyatomic second population: Eq. (eq:discrete-equilibrium-poly);
 *   - Knudsen sensor: Eq. (eq:DeltaAvg); relaxation factor: Eq. (eq:alpha);
 *   - BGK collide-and-stream for h = f, g with Pr = 1: Sec. 3;
 *   - free-stream equilibrium faces, first-order Neumann outlet and half-way
 *     bounce-back: Sec. 4 (NACA0012 set-up).
 * Readings where the paper is silent or garbled are marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 39   /* discrete velocities */
#define NL 13   /* Lagrange multipliers / constraints */
#define DIM 3   /* the lattice is three-dimensional for every grid */

/* ------------------------------------------------------------------------ */
/* Lattice (Sec. 3): (0,0,0), (1,0,0)_FS, (+-1,+-1,+-1), (2,0,0)_FS,          */
/* (2,2,0)_FS, (3,0,0)_FS.  Listed so that for every odd i, velocity i+1 is   */
/* the opposite of velocity i (an interface convention of the library).       */
/* ------------------------------------------------------------------------ */
static const int VEL[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
    {-1, 1, 1},  {1, -1, -1},
    {2, 0, 0},   {-2, 0, 0},  {0, 2, 0},   {0, -2, 0},  {0, 0, 2},   {0, 0, -2},
    {2, 2, 0},   {-2, -2, 0}, {2, -2, 0},  {-2, 2, 0},  {2, 0, 2},   {-2, 0, -2},
    {2, 0, -2},  {-2, 0, 2},  {0, 2, 2},   {0, -2, -2}, {0, 2, -2},  {0, -2, 2},
    {3, 0, 0},   {-3, 0, 0},  {0, 3, 0},   {0, -3, 0},  {0, 0, 3},   {0, 0, -3},
};

static int opposite(int i)
{
    int j;
    for (j = 0; j < NQ; ++j)
        if (VEL[j][0] == -VEL[i][0] && VEL[j][1] == -VEL[i][1] && VEL[j][2] == -VEL[i][2])
            return j;
    return -1;
}

/* Basis of the 13-moment exponent, Eq. (eq:discrete-equilibrium):
 * 1, xi_a (3), xi_a xi_b for a <= b (6), xi_a |xi|^2 (3).  The multiplier of
 * the off-diagonal product xi_a xi_b absorbs the factor 2 of the symmetric
 * double sum; only f^eq is observable, so the parameterisation is free. */
static void basis(const double c[3], double phi[NL])
{
    double q = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    phi[0] = 1.0;
    phi[1] = c[0];
    phi[2] = c[1];
    phi[3] = c[2];
    phi[4] = c[0] * c[0];
    phi[5] = c[1] * c[1];
    phi[6] = c[2] * c[2];
    phi[7] = c[0] * c[1];
    phi[8] = c[0] * c[2];
    phi[9] = c[1] * c[2];
    phi[10] = c[0] * q;
    phi[11] = c[1] * q;
    phi[12] = c[2] * q;
}

static double PHI[NQ][NL];
static int OPP[NQ];
static int tables_ready = 0;

static void make_tables(void)
{
    int i;
    if (tables_ready) return;
    for (i = 0; i < NQ; ++i) {
        double c[3] = {VEL[i][0], VEL[i][1], VEL[i][2]};
        basis(c, PHI[i]);
        OPP[i] = opposite(i);
    }
    tables_ready = 1;
}

/* Maxwell-Boltzmann moments per unit density, Eq. (eq:EqMomentsTensor),
 * restricted to the 13 constraints of Eq. (eq:13constraints).
 * Reading: the contracted third moment is sum_b M3_abb = rho u_a (|u|^2 +
 * (D+2) T), which is what contracting the printed third-order tensor gives;
 * the printed "E^tr = D T + rho u^2" is dimensionally garbled. */
static void mb_targets(const double u[3], double T, double m[NL])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double h = uu + (DIM + 2) * T;
    m[0] = 1.0;
    m[1] = u[0];
    m[2] = u[1];
    m[3] = u[2];
    m[4] = u[0] * u[0] + T;
    m[5] = u[1] * u[1] + T;
    m[6] = u[2] * u[2] + T;
    m[7] = u[0] * u[1];
    m[8] = u[0] * u[2];
    m[9] = u[1] * u[2];
    m[10] = h * u[0];
    m[11] = h * u[1];
    m[12] = h * u[2];
}

/* f^eq_i / rho = exp(phi_i . lambda) for the current multipliers, and the
 * constraint residual G = sum_i f^eq_i phi_i / rho - M/rho, Eq. (eq:constraints). */
static void equilibrium_and_residual(const double lam[NL], const double m[NL], double feq[NQ], double G[NL])
{
    int i, k;
    for (i = 0; i < NQ; ++i) {
        double e = 0.0;
        for (k = 0; k < NL; ++k) e += PHI[i][k] * lam[k];
        feq[i] = exp(e);
    }
    for (k = 0; k < NL; ++k) {
        double s = 0.0;
        for (i = 0; i < NQ; ++i) s += feq[i] * PHI[i][k];
        G[k] = s - m[k];
    }
}

/* Jacobian of G with respect to lambda: J_kl = sum_i f^eq_i phi_ik phi_il. */
static void jacobian(const double feq[NQ], double J[NL][NL])
{
    int i, k, l;
    for (k = 0; k < NL; ++k)
        for (l = 0; l < NL; ++l) {
            double s = 0.0;
            for (i = 0; i < NQ; ++i) s += feq[i] * PHI[i][k] * PHI[i][l];
            J[k][l] = s;
        }
}

/* Solve J d = G.  The paper inverts J; J is symmetric positive definite
 * (a Gram matrix of 13 linearly independent functions on 39 velocities), so a
 * Cholesky solve gives the same d.  Returns 0 on success. */
static int cholesky_solve(double J[NL][NL], const double G[NL], double d[NL])
{
    double L[NL][NL];
    double y[NL];
    int i, j, k;
    memset(L, 0, sizeof(L));
    for (j = 0; j < NL; ++j) {
        double s = J[j][j];
        for (k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0)) return -1;
        L[j][j] = sqrt(s);
        for (i = j + 1; i < NL; ++i) {
            double t = J[i][j];
            for (k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    for (i = 0; i < NL; ++i) {
        double t = G[i];
        for (k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    for (i = NL - 1; i >= 0; --i) {
        double t = y[i];
        for (k = i + 1; k < NL; ++k) t -= L[k][i] * d[k];
        d[i] = t / L[i][i];
    }
    return 0;
}

static double norm_inf(const double v[NL])
{
    double r = 0.0;
    int k;
    for (k = 0; k < NL; ++k) {
        double a = fabs(v[k]);
        if (!(a <= r)) r = a; /* NaN propagates */
    }
    return r;
}

static double norm_2(const double v[NL])
{
    double r = 0.0;
    int k;
    for (k = 0; k < NL; ++k) r += v[k] * v[k];
    return sqrt(r);
}

/* lambda_0 that normalises sum_i exp(phi_i . lambda) to 1 for the other 12
 * multipliers. */
static void normalise(double lam[NL])
{
    double s = 0.0;
    int i, k;
    for (i = 0; i < NQ; ++i) {
        double e = 0.0;
        for (k = 1; k < NL; ++k) e += PHI[i][k] * lam[k];
        s += exp(e);
    }
    lam[0] = -log(s);
}

/* Cold start of the multipliers at t = 0 (reading: the paper only gives the
 * warm start from t - 1): the Maxwellian shape lambda_1 = u/T,
 * lambda_2 = -delta/(2T), lambda_3 = 0, lambda_0 normalising the sum to 1. */
static void cold_guess(const double u[3], double T, double lam[NL])
{
    int k;
    for (k = 0; k < NL; ++k) lam[k] = 0.0;
    lam[1] = u[0] / T;
    lam[2] = u[1] / T;
    lam[3] = u[2] / T;
    lam[4] = lam[5] = lam[6] = -0.5 / T;
    normalise(lam);
}

/* Newton-Raphson for the 13 multipliers (Sec. 5 algorithm table): evaluate
 * f^eq and G; stop when the error norm is below tol; otherwise build J, solve,
 * and step.  Reading of the stopping norm: max_k |G_k| / rho <=
 * tol * max(1, max_k |M_k| / rho).  Globalisation (reading; the paper says
 * only "standard multivariate Newton-Raphson"): the step is halved while the
 * Euclidean norm of G does not decrease, trying t = 1, 1/2, ..., 2^-39.
 * Round-off floor (reading, switch floor_rule): if the full step does not
 * lower the norm while max_k |G_k| before and after it is within 8 times the
 * bound, the step is taken and the solve stops.  Stall (reading): when no
 * trial lowers the norm, the attempt fails (no descent is left along the
 * Newton direction, which happens where no multipliers satisfy the
 * constraints).  On return lam and feq (per unit density) hold the last
 * iterate and *evals (if not NULL) has been increased by the number of f^eq
 * evaluations.  Returns the number of accepted updates, or -1 when the cap
 * is reached, J is not positive definite, a value is not finite, or the line
 * search stalls. */
static int newton(const double m[NL], double lam[NL], double feq[NQ], double tol, int maxit, int floor_rule,
                  int64_t *evals)
{
    double G[NL], J[NL][NL], d[NL], trial[NL], Gt[NL], ft[NQ];
    double scale = 1.0;
    int it, k, ls;
    int64_t ne = 1;
    for (k = 0; k < NL; ++k)
        if (fabs(m[k]) > scale) scale = fabs(m[k]);
    equilibrium_and_residual(lam, m, feq, G);
    for (it = 0;; ++it) {
        double r = norm_inf(G);
        double n0, t = 1.0;
        int descended = 0;
        if (!isfinite(r)) break;
        if (r <= tol * scale) {
            if (evals) *evals += ne;
            return it;
        }
        if (it >= maxit) break;
        jacobian(feq, J);
        if (cholesky_solve(J, G, d) != 0) break;
        n0 = norm_2(G);
        for (ls = 0; ls < 40; ++ls) {
            for (k = 0; k < NL; ++k) trial[k] = lam[k] - t * d[k];
            equilibrium_and_residual(trial, m, ft, Gt);
            ne += 1;
            if (norm_2(Gt) < n0) {
                descended = 1;
                break;
            }
            if (ls == 0 && floor_rule && r <= 8.0 * tol * scale && norm_inf(Gt) <= 8.0 * tol * scale) {
                /* the residual sits at the round-off floor of the arithmetic */
                for (k = 0; k < NL; ++k) lam[k] = trial[k];
                for (k = 0; k < NQ; ++k) feq[k] = ft[k];
                if (evals) *evals += ne;
                return it + 1;
            }
            t *= 0.5;
        }
        if (!descended) break;
        for (k = 0; k < NL; ++k) {
            lam[k] = trial[k];
            G[k] = Gt[k];
        }
        for (k = 0; k < NQ; ++k) feq[k] = ft[k];
    }
    if (evals) *evals += ne;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Variant of the root finder (Sec. 6 names the choice between gradient-based */
/* and gradient-free algorithms as an open question): a secant method that   */
/* never evaluates the Jacobian of G.                                         */
/* ------------------------------------------------------------------------ */

/* Powers of the basis functions in xi: 0 for 1, 1 for xi_a, 2 for the
 * products, 3 for xi_a |xi|^2. */
static const int BASIS_DEGREE[NL] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3};

/* A(v) with phi(xi + v) = A(v) phi(xi) for every xi: the span of the 13 basis
 * functions is closed under shifts of xi (the shift of xi_a |xi|^2 stays a
 * polynomial of degree 3 whose cubic part is xi_a |xi|^2 again).  Built from
 * that definition: on the 39 velocities Phi (39 x 13) has rank 13, so
 * A(v)^T = (Phi^T Phi)^-1 Phi^T Phi_v with Phi_v[i][k] = phi_k(xi_i + v). */
static void shift_matrix(const double v[3], double A[NL][NL])
{
    double M[NL][NL], col[NL], x[NL];
    double Pv[NQ][NL];
    int i, k, l;
    for (i = 0; i < NQ; ++i) {
        double c[3] = {VEL[i][0] + v[0], VEL[i][1] + v[1], VEL[i][2] + v[2]};
        basis(c, Pv[i]);
    }
    for (k = 0; k < NL; ++k)
        for (l = 0; l < NL; ++l) {
            double t = 0.0;
            for (i = 0; i < NQ; ++i) t += PHI[i][k] * PHI[i][l];
            M[k][l] = t;
        }
    for (l = 0; l < NL; ++l) {  /* column l of A^T is row l of A */
        double Mc[NL][NL];
        for (k = 0; k < NL; ++k) {
            double t = 0.0;
            for (i = 0; i < NQ; ++i) t += PHI[i][k] * Pv[i][l];
            col[k] = t;
        }
        memcpy(Mc, M, sizeof(M));
        cholesky_solve(Mc, col, x);
        for (k = 0; k < NL; ++k) A[l][k] = x[k];
    }
}

/* Model of the Jacobian at (u, T): J_model = A(u) D J_rest D A(u)^T with
 * D = diag((T / T_ref)^(degree_k / 2)).  For the continuous Maxwellian this
 * is exact: its moment matrix E[phi phi^T] at (u, T) is that of rest at T_ref
 * with xi scaled by sqrt(T / T_ref) and shifted by u.  J_rest is the Jacobian
 * at the lattice's own rest equilibrium at T_ref, so at u = 0, T = T_ref the
 * model is the true Jacobian there. */
static void model_jacobian(const double u[3], double T, double T_ref, const double Jrest[NL][NL], double Jm[NL][NL])
{
    double A[NL][NL], B[NL][NL], Dg[NL];
    int k, l, a;
    shift_matrix(u, A);
    for (k = 0; k < NL; ++k) Dg[k] = pow(T / T_ref, 0.5 * BASIS_DEGREE[k]);
    /* B = A D J_rest D */
    for (k = 0; k < NL; ++k)
        for (l = 0; l < NL; ++l) {
            double t = 0.0;
            for (a = 0; a < NL; ++a) t += A[k][a] * Dg[a] * Jrest[a][l] * Dg[l];
            B[k][l] = t;
        }
    for (k = 0; k < NL; ++k)
        for (l = 0; l < NL; ++l) {
            double t = 0.0;
            for (a = 0; a < NL; ++a) t += B[k][a] * A[l][a];
            Jm[k][l] = t;
        }
}

/* Jacobian of the lattice's rest equilibrium at temperature T_ref (per unit
 * density), the equilibrium found by this file's Newton from the cold guess. */
static int rest_jacobian(double T_ref, double Jrest[NL][NL])
{
    double m[NL], lam[NL], feq[NQ];
    const double u0[3] = {0.0, 0.0, 0.0};
    mb_targets(u0, T_ref, m);
    cold_guess(u0, T_ref, lam);
    if (newton(m, lam, feq, 1e-15, 100, 1, NULL) < 0) return -1;
    jacobian(feq, Jrest);
    return 0;
}

#define SECANT_MEMORY 3

/* Limited-memory BFGS (Nocedal and Wright, Numerical Optimization, the
 * two-loop recursion) for G(lambda) = 0, G being the gradient of the convex
 * dual Phi(lambda) = sum_i exp(phi_i . lambda) - lambda . m, so that J is
 * Phi's Hessian.  Only residuals G are evaluated: the direction d = H G uses
 * the last SECANT_MEMORY pairs s = lambda_new - lambda_old, y = G_new - G_old
 * (kept only when s . y > 0) on top of H0 = J_model^-1 (model_jacobian).  The
 * step is lambda - t d, t = 1, 1/2, ..., 2^-39; a trial is accepted when it
 * lowers the Euclidean norm of G (the Newton rule) or, for a descent
 * direction (G . d > 0), when it lowers Phi by at least 1e-4 t G . d
 * (Armijo), which a positive definite H guarantees for small t.  Stopping
 * rule, round-off floor stop (floor_rule) and stall as in newton().  Returns
 * the number of accepted updates, or -1 (cap, stall, value not finite). */
static int secant(const double m[NL], double lam[NL], double feq[NQ], double tol, int maxit, int floor_rule,
                  const double Jm[NL][NL], int64_t *evals)
{
    double G[NL], Gt[NL], ft[NQ], trial[NL], d[NL];
    double S[SECANT_MEMORY][NL], Y[SECANT_MEMORY][NL], rho_s[SECANT_MEMORY];
    double scale = 1.0, phi, lm;
    int it, k, ls, np = 0;
    int64_t ne = 1;
    for (k = 0; k < NL; ++k)
        if (fabs(m[k]) > scale) scale = fabs(m[k]);
    equilibrium_and_residual(lam, m, feq, G);
    phi = 0.0;
    for (k = 0; k < NQ; ++k) phi += feq[k];
    lm = 0.0;
    for (k = 0; k < NL; ++k) lm += lam[k] * m[k];
    phi -= lm;
    for (it = 0;; ++it) {
        double r = norm_inf(G);
        double n0, gd, t = 1.0, q[NL], al[SECANT_MEMORY];
        double Jc[NL][NL];
        int j, accepted = 0;
        if (!isfinite(r)) break;
        if (r <= tol * scale) {
            if (evals) *evals += ne;
            return it;
        }
        if (it >= maxit) break;
        /* two-loop recursion: d = H G */
        for (k = 0; k < NL; ++k) q[k] = G[k];
        for (j = np - 1; j >= 0; --j) {
            double t2 = 0.0;
            for (k = 0; k < NL; ++k) t2 += S[j][k] * q[k];
            al[j] = rho_s[j] * t2;
            for (k = 0; k < NL; ++k) q[k] -= al[j] * Y[j][k];
        }
        memcpy(Jc, Jm, sizeof(Jc));
        if (cholesky_solve(Jc, q, d) != 0) break;
        for (j = 0; j < np; ++j) {
            double b = 0.0;
            for (k = 0; k < NL; ++k) b += Y[j][k] * d[k];
            b *= rho_s[j];
            for (k = 0; k < NL; ++k) d[k] += S[j][k] * (al[j] - b);
        }
        n0 = norm_2(G);
        gd = 0.0;
        for (k = 0; k < NL; ++k) gd += G[k] * d[k];
        for (ls = 0; ls < 40; ++ls) {
            double pt = 0.0;
            for (k = 0; k < NL; ++k) trial[k] = lam[k] - t * d[k];
            equilibrium_and_residual(trial, m, ft, Gt);
            ne += 1;
            for (k = 0; k < NQ; ++k) pt += ft[k];
            lm = 0.0;
            for (k = 0; k < NL; ++k) lm += trial[k] * m[k];
            pt -= lm;
            if (norm_2(Gt) < n0 || (gd > 0.0 && pt <= phi - 1e-4 * t * gd)) {
                accepted = 1;
                phi = pt;
                break;
            }
            if (ls == 0 && floor_rule && r <= 8.0 * tol * scale && norm_inf(Gt) <= 8.0 * tol * scale) {
                for (k = 0; k < NL; ++k) lam[k] = trial[k];
                for (k = 0; k < NQ; ++k) feq[k] = ft[k];
                if (evals) *evals += ne;
                return it + 1;
            }
            t *= 0.5;
        }
        if (!accepted) break;
        {
            double sv[NL], yv[NL], sy = 0.0;
            for (k = 0; k < NL; ++k) {
                sv[k] = -t * d[k];  /* the step taken */
                yv[k] = Gt[k] - G[k];
                sy += sv[k] * yv[k];
            }
            if (sy > 0.0) {
                if (np == SECANT_MEMORY) {
                    for (j = 1; j < SECANT_MEMORY; ++j) {
                        memcpy(S[j - 1], S[j], sizeof(S[j]));
                        memcpy(Y[j - 1], Y[j], sizeof(Y[j]));
                        rho_s[j - 1] = rho_s[j];
                    }
                    np -= 1;
                }
                memcpy(S[np], sv, sizeof(sv));
                memcpy(Y[np], yv, sizeof(yv));
                rho_s[np] = 1.0 / sy;
                np += 1;
            }
        }
        for (k = 0; k < NL; ++k) {
            lam[k] = trial[k];
            G[k] = Gt[k];
        }
        for (k = 0; k < NQ; ++k) feq[k] = ft[k];
    }
    if (evals) *evals += ne;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Public interface (ctypes)                                                */
/* ------------------------------------------------------------------------ */

enum { FACE_PERIODIC = 0, FACE_EQUILIBRIUM = 1, FACE_NEUMANN = 2 };
enum { CELL_FLUID = 0, CELL_SOLID = 1, CELL_FROZEN = 2, CELL_NEUMANN = 3 };

typedef struct {
    int32_t nx, ny, nz;
    int32_t kn_relax;      /* 1: tau * alpha(eps), Eq. (eq:alpha); 0: plain BGK */
    int32_t newton_maxit;
    int32_t faces[6];      /* -x, +x, -y, +y, -z, +z */
    double gamma;          /* C_v = 1/(gamma - 1) */
    double tau;
    double newton_tol;
    const uint8_t *solid;  /* nx*ny*nz or NULL */
    /* readings that the pins switch off to show what they change (1 = on) */
    int32_t floor_rule;    /* stop at the round-off floor (see newton) */
    int32_t skip_cold_after_failure; /* a cell that failed the previous step is not restarted cold */
    int32_t root_finder;   /* 0: Newton-Raphson (the paper's); 1: the secant variant */
    double model_T;        /* root_finder 1: temperature of the rest Jacobian of its model */
} orc_params;

typedef struct {
    int64_t iterations;    /* accepted Newton updates, summed over fluid cells */
    int64_t max_iterations;
    int64_t failed;        /* cells whose Newton did not converge */
    int64_t alpha_hist[4]; /* cells per branch of Eq. (eq:alpha) */
    int64_t cold_restarts; /* cells that fell back to the cold start */
    int64_t evaluations;   /* f^eq evaluations of the Newton solves (line-search trials included) */
} orc_stats;

void orc_velocities(int32_t *out)
{
    int i;
    for (i = 0; i < NQ; ++i) {
        out[3 * i + 0] = VEL[i][0];
        out[3 * i + 1] = VEL[i][1];
        out[3 * i + 2] = VEL[i][2];
    }
}

static double heat_capacity(double gamma) { return 1.0 / (gamma - 1.0); }

/* Equilibrium of one cell: returns iterations (or -1); writes lam (in/out:
 * used as the warm start unless cold != 0) and f^eq, g^eq (not per unit
 * density).  g^eq = (2 C_v - D) T f^eq, Eq. (eq:discrete-equilibrium-poly). */
int orc_equilibrium(double rho, const double *u, double T, double gamma, double *lam, int cold, double tol,
                    int maxit, double *feq_out, double *geq_out)
{
    double m[NL], feq[NQ];
    double delta = 2.0 * heat_capacity(gamma) - DIM;
    int it, i;
    make_tables();
    mb_targets(u, T, m);
    if (cold) cold_guess(u, T, lam);
    it = newton(m, lam, feq, tol, maxit, 1, NULL);
    for (i = 0; i < NQ; ++i) {
        if (feq_out) feq_out[i] = rho * feq[i];
        if (geq_out) geq_out[i] = delta * T * rho * feq[i];
    }
    return it;
}

static int64_t cell_index(const orc_params *p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

static int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Cell classification.  Reading of the face conditions with a three-cell
 * reach: the three outermost layers of a non-periodic face are boundary
 * cells.  Equilibrium faces hold the equilibrium of their initial state and
 * are never updated; Neumann faces copy the nearest interior cell before each
 * step (first-order zero gradient).  Equilibrium takes precedence where an
 * equilibrium face and a Neumann face meet. */
static int in_face_layer(const orc_params *p, int x, int y, int z, int kind)
{
    int n[3] = {p->nx, p->ny, p->nz};
    int c[3] = {x, y, z};
    int a;
    for (a = 0; a < 3; ++a) {
        if (p->faces[2 * a] == kind && c[a] < 3) return 1;
        if (p->faces[2 * a + 1] == kind && c[a] >= n[a] - 3) return 1;
    }
    return 0;
}

static int cell_type(const orc_params *p, int x, int y, int z)
{
    if (p->solid && p->solid[cell_index(p, x, y, z)]) return CELL_SOLID;
    if (in_face_layer(p, x, y, z, FACE_EQUILIBRIUM)) return CELL_FROZEN;
    if (in_face_layer(p, x, y, z, FACE_NEUMANN)) return CELL_NEUMANN;
    return CELL_FLUID;
}

void orc_cell_types(const orc_params *p, uint8_t *out)
{
    int x, y, z;
    for (z = 0; z < p->nz; ++z)
        for (y = 0; y < p->ny; ++y)
            for (x = 0; x < p->nx; ++x) out[cell_index(p, x, y, z)] = (uint8_t)cell_type(p, x, y, z);
}

/* The cell whose populations a Neumann boundary cell copies: its coordinates
 * clamped into the interior along every Neumann axis. */
static int64_t neumann_source(const orc_params *p, int x, int y, int z)
{
    int n[3] = {p->nx, p->ny, p->nz};
    int c[3] = {x, y, z};
    int a;
    for (a = 0; a < 3; ++a) {
        if (p->faces[2 * a] == FACE_NEUMANN && c[a] < 3) c[a] = 3;
        if (p->faces[2 * a + 1] == FACE_NEUMANN && c[a] >= n[a] - 3) c[a] = n[a] - 4;
    }
    return cell_index(p, c[0], c[1], c[2]);
}

/* Neighbour coordinate along one axis: periodic axes wrap; on other axes the
 * three boundary layers guarantee that interior cells stay inside. */
static int step_axis(const orc_params *p, int a, int c, int d)
{
    int n = a == 0 ? p->nx : (a == 1 ? p->ny : p->nz);
    int lo = p->faces[2 * a], hi = p->faces[2 * a + 1];
    if (lo == FACE_PERIODIC && hi == FACE_PERIODIC) return wrap(c + d, n);
    return c + d;
}

/* Primitive direction and multiplicity of a velocity: xi = mult * dir. */
static int multiplicity(int i)
{
    int a, g = 0;
    for (a = 0; a < 3; ++a) {
        int v = abs(VEL[i][a]);
        if (v > g) g = v;
    }
    /* every D3Q39 velocity is a multiple of a vector with entries in {-1,0,1} */
    return g;
}

/* Pull streaming of population i into fluid cell (x,y,z) (the push form of
 * Sec. 3 written as a gather).  Half-way bounce-back for multi-speed links
 * (reading; the paper states half-way bounce-back only): the link is blocked
 * when any lattice node passed over, x - k dir_i for k = 1..mult_i, is
 * solid; the cell then receives its own post-collision population of the
 * opposite direction. */
static int64_t pull_source(const orc_params *p, int x, int y, int z, int i, int *bounced)
{
    int m = multiplicity(i);
    int d[3], k, a;
    int c[3] = {x, y, z};
    for (a = 0; a < 3; ++a) d[a] = VEL[i][a] / (m == 0 ? 1 : m);
    *bounced = 0;
    if (m == 0) return cell_index(p, x, y, z);
    if (p->solid) {
        for (k = 1; k <= m; ++k) {
            int s[3];
            for (a = 0; a < 3; ++a) s[a] = step_axis(p, a, c[a], -k * d[a]);
            if (p->solid[cell_index(p, s[0], s[1], s[2])]) {
                *bounced = 1;
                return cell_index(p, x, y, z);
            }
        }
    }
    {
        /* Reading of the Neumann rule: a coordinate inside a Neumann face's
         * three layers reads the nearest interior layer along that face's
         * normal, also where the layer meets another face. */
        int s[3];
        for (a = 0; a < 3; ++a) s[a] = step_axis(p, a, c[a], -VEL[i][a]);
        return neumann_source(p, s[0], s[1], s[2]);
    }
}

/* Macroscopic variables of one cell from its populations (Sec. 3 and the
 * first row of the Sec. 5 table).  Reading (the paper does not write T out):
 * total energy 2 rho E = sum f |xi|^2 + sum g, with E = |u|^2/2 + C_v T
 * (equation of state under Eq. (eq:NSF)). */
static void macroscopic(const double f[NQ], const double g[NQ], double gamma, double *rho, double u[3], double *T)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0}, e = 0.0, uu;
    int i, a;
    for (i = 0; i < NQ; ++i) {
        r += f[i];
        for (a = 0; a < 3; ++a) j[a] += f[i] * VEL[i][a];
        e += f[i] * (VEL[i][0] * VEL[i][0] + VEL[i][1] * VEL[i][1] + VEL[i][2] * VEL[i][2]);
        e += g[i];
    }
    for (a = 0; a < 3; ++a) u[a] = j[a] / r;
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    *rho = r;
    *T = (e - r * uu) / (2.0 * heat_capacity(gamma) * r);
}

/* Relaxation factor alpha(eps) of Eq. (eq:alpha); intervals closed on the
 * left as printed.  Returns the branch index 0..3. */
static int alpha_branch(double eps)
{
    if (eps < 1e-2) return 0;
    if (eps < 1e-1) return 1;
    if (eps < 1.0) return 2;
    return 3; /* also NaN/inf: the cell is replaced by its equilibrium */
}

/* Initial state: every cell holds the equilibrium of its (rho, u, T) field,
 * computed with the cold start; the multipliers are stored for the warm start.
 * Returns the number of cells whose Newton did not converge. */
/* The secant variant for one cell: as orc_equilibrium, with the model
 * Jacobian built on the rest equilibrium at T_ref.  Returns the number of
 * accepted updates or -1. */
int orc_equilibrium_secant(double rho, const double *u, double T, double T_ref, double gamma, double *lam, int cold,
                           double tol, int maxit, double *feq_out, double *geq_out)
{
    double m[NL], feq[NQ], Jrest[NL][NL], Jm[NL][NL];
    double delta = 2.0 * heat_capacity(gamma) - DIM;
    int it, i;
    make_tables();
    if (rest_jacobian(T_ref, Jrest) != 0) return -2;
    model_jacobian(u, T, T_ref, (const double(*)[NL])Jrest, Jm);
    mb_targets(u, T, m);
    if (cold) cold_guess(u, T, lam);
    it = secant(m, lam, feq, tol, maxit, 1, (const double(*)[NL])Jm, NULL);
    for (i = 0; i < NQ; ++i) {
        if (feq_out) feq_out[i] = rho * feq[i];
        if (geq_out) geq_out[i] = delta * T * rho * feq[i];
    }
    return it;
}

/* The secant variant's model Jacobian at (u, T) (row-major 13 x 13) built
 * on Jrest_in (row-major, or NULL for the lattice's rest Jacobian at T_ref),
 * and the shift matrix A(u) of phi(xi + u) = A(u) phi(xi). */
int orc_model_jacobian(const double *u, double T, double T_ref, const double *Jrest_in, double *J_out, double *A_out)
{
    double Jrest[NL][NL], Jm[NL][NL], A[NL][NL];
    int k, l;
    make_tables();
    if (Jrest_in) {
        for (k = 0; k < NL; ++k)
            for (l = 0; l < NL; ++l) Jrest[k][l] = Jrest_in[k * NL + l];
    } else if (rest_jacobian(T_ref, Jrest) != 0) {
        return -1;
    }
    model_jacobian(u, T, T_ref, (const double(*)[NL])Jrest, Jm);
    shift_matrix(u, A);
    for (k = 0; k < NL; ++k)
        for (l = 0; l < NL; ++l) {
            if (J_out) J_out[k * NL + l] = Jm[k][l];
            if (A_out) A_out[k * NL + l] = A[k][l];
        }
    return 0;
}

int64_t orc_init(const orc_params *p, const double *rho, const double *u, const double *T, double *f, double *g,
                 double *lam)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    int64_t c, failed = 0;
    make_tables();
#pragma omp parallel for reduction(+ : failed) schedule(dynamic, 64)
    for (c = 0; c < n; ++c) {
        double uc[3] = {u[c], u[n + c], u[2 * n + c]};
        double l[NL], fe[NQ], ge[NQ];
        int i, k, maxit = p->newton_maxit > 100 ? p->newton_maxit : 100;
        int it = orc_equilibrium(rho[c], uc, T[c], p->gamma, l, 1, p->newton_tol, maxit, fe, ge);
        if (it < 0) failed += 1;
        for (i = 0; i < NQ; ++i) {
            f[i * n + c] = fe[i];
            g[i * n + c] = ge[i];
        }
        for (k = 0; k < NL; ++k) lam[k * n + c] = l[k];
    }
    return failed;
}

/* One time step: for every fluid cell, stream (pull), compute the
 * macroscopic variables, the Maxwell-Boltzmann targets, the multipliers by
 * Newton from the stored ones, f^eq and g^eq, the Knudsen sensor and the
 * relaxation factor, and write the BGK-relaxed populations.  Boundary and
 * solid cells are copied unchanged.  A fluid cell whose Newton solve fails
 * (warm start, then cold start) is not collided: its gathered populations are
 * written unchanged and its multipliers kept, with lambda_0 replaced by NaN
 * as the mark of the failure; it is counted in st->failed and in no alpha
 * branch.  A marked cell warm-starts from its other 12 multipliers
 * (lambda_0 normalising) and, with skip_cold_after_failure, is not restarted
 * cold.  iters_out / eps_out (length N, or NULL) receive per-cell
 * diagnostics (-1 / NaN outside fluid cells, NaN for eps of a failed cell). */
void orc_step(const orc_params *p, const double *f, const double *g, const double *lam, double *fo, double *go,
              double *lamo, int32_t *iters_out, double *eps_out, orc_stats *st)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    int64_t c;
    int64_t s_it = 0, s_max = 0, s_fail = 0, s_cold = 0, h0 = 0, h1 = 0, h2 = 0, h3 = 0, s_ev = 0;
    double Cv = heat_capacity(p->gamma);
    double delta = 2.0 * Cv - DIM;
    double Jrest[NL][NL];
    make_tables();
    if (p->root_finder == 1 && rest_jacobian(p->model_T, Jrest) != 0) return;
#pragma omp parallel for schedule(dynamic, 64) \
    reduction(+ : s_it, s_fail, s_cold, h0, h1, h2, h3, s_ev) reduction(max : s_max)
    for (c = 0; c < n; ++c) {
        int x = (int)(c % p->nx);
        int y = (int)((c / p->nx) % p->ny);
        int z = (int)(c / ((int64_t)p->nx * p->ny));
        int i, k, it, br, bounced, marked;
        double fi[NQ], gi[NQ], l[NL], m[NL], feq[NQ], geq[NQ];
        double rho, u[3], T, eps, tau_eff, omega;
        double Jm[NL][NL];
        if (cell_type(p, x, y, z) != CELL_FLUID) {
            for (i = 0; i < NQ; ++i) {
                fo[i * n + c] = f[i * n + c];
                go[i * n + c] = g[i * n + c];
            }
            for (k = 0; k < NL; ++k) lamo[k * n + c] = lam[k * n + c];
            if (iters_out) iters_out[c] = -1;
            if (eps_out) eps_out[c] = NAN;
            continue;
        }
        /* streaming */
        for (i = 0; i < NQ; ++i) {
            int64_t s = pull_source(p, x, y, z, i, &bounced);
            int src_pop = bounced ? OPP[i] : i;
            fi[i] = f[src_pop * n + s];
            gi[i] = g[src_pop * n + s];
        }
        /* macroscopic variables and targets */
        macroscopic(fi, gi, p->gamma, &rho, u, &T);
        mb_targets(u, T, m);
        /* multipliers: warm start from the previous step */
        for (k = 0; k < NL; ++k) l[k] = lam[k * n + c];
        marked = isnan(l[0]);
        if (marked) normalise(l);
        if (p->root_finder == 1) {
            model_jacobian(u, T, p->model_T, (const double(*)[NL])Jrest, Jm);
            it = secant(m, l, feq, p->newton_tol, p->newton_maxit, p->floor_rule, (const double(*)[NL])Jm, &s_ev);
        } else {
            it = newton(m, l, feq, p->newton_tol, p->newton_maxit, p->floor_rule, &s_ev);
        }
        if (it < 0) {
            /* reading: a failed warm start is retried once from the cold
             * start before the cell is counted as failed, unless the cell
             * also failed the previous step (then the retry is skipped, which
             * bounds the cost of a cell that has no equilibrium) */
            int it2 = -1;
            if (!(marked && p->skip_cold_after_failure)) {
                s_cold += 1;
                cold_guess(u, T, l);
                if (p->root_finder == 1)
                    it2 = secant(m, l, feq, p->newton_tol, p->newton_maxit > 100 ? p->newton_maxit : 100,
                                 p->floor_rule, (const double(*)[NL])Jm, &s_ev);
                else
                    it2 = newton(m, l, feq, p->newton_tol, p->newton_maxit > 100 ? p->newton_maxit : 100,
                                 p->floor_rule, &s_ev);
            }
            if (it2 < 0) {
                /* reading: where no multipliers reproduce the 13 targets the
                 * cell is not collided; its gathered populations are stored
                 * as they are and its multipliers are kept (the paper gives
                 * no rule; this one conserves every moment of the cell) */
                s_fail += 1;
                s_it += p->newton_maxit;
                if (p->newton_maxit > s_max) s_max = p->newton_maxit;
                for (i = 0; i < NQ; ++i) {
                    fo[i * n + c] = fi[i];
                    go[i * n + c] = gi[i];
                }
                for (k = 0; k < NL; ++k) lamo[k * n + c] = lam[k * n + c];
                lamo[c] = NAN;
                if (iters_out) iters_out[c] = p->newton_maxit;
                if (eps_out) eps_out[c] = NAN;
                continue;
            }
            it = it2;
        }
        s_it += it;
        if (it > s_max) s_max = it;
        for (i = 0; i < NQ; ++i) {
            feq[i] *= rho;
            geq[i] = delta * T * feq[i];
        }
        /* Knudsen sensor over f only, Eq. (eq:DeltaAvg) */
        eps = 0.0;
        for (i = 0; i < NQ; ++i) eps += fabs(fi[i] - feq[i]) / feq[i];
        eps /= NQ;
        br = p->kn_relax ? alpha_branch(eps) : 0;
        if (br == 0) h0 += 1;
        else if (br == 1) h1 += 1;
        else if (br == 2) h2 += 1;
        else h3 += 1;
        /* tau(eps) = tau * alpha(eps); alpha = 1/tau gives tau_eff = 1 */
        if (br == 0) tau_eff = p->tau;
        else if (br == 1) tau_eff = p->tau * 1.05;
        else if (br == 2) tau_eff = p->tau * 1.35;
        else tau_eff = 1.0;
        omega = 1.0 / tau_eff;
        /* BGK, the same relaxation time for f and g (Pr = 1) */
        for (i = 0; i < NQ; ++i) {
            fo[i * n + c] = fi[i] + omega * (feq[i] - fi[i]);
            go[i * n + c] = gi[i] + omega * (geq[i] - gi[i]);
        }
        for (k = 0; k < NL; ++k) lamo[k * n + c] = l[k];
        if (iters_out) iters_out[c] = it;
        if (eps_out) eps_out[c] = eps;
    }
    if (st) {
        st->iterations = s_it;
        st->max_iterations = s_max;
        st->failed = s_fail;
        st->cold_restarts = s_cold;
        st->evaluations = s_ev;
        st->alpha_hist[0] = h0;
        st->alpha_hist[1] = h1;
        st->alpha_hist[2] = h2;
        st->alpha_hist[3] = h3;
    }
}

/* Pure streaming (no collision) of one population array, with the same
 * boundary rules as orc_step; used to check that the gather is a permutation. */
void orc_stream_only(const orc_params *p, const double *f, double *fo)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    int64_t c;
    make_tables();
    for (c = 0; c < n; ++c) {
        int x = (int)(c % p->nx);
        int y = (int)((c / p->nx) % p->ny);
        int z = (int)(c / ((int64_t)p->nx * p->ny));
        int i, bounced;
        for (i = 0; i < NQ; ++i) {
            if (cell_type(p, x, y, z) != CELL_FLUID) {
                fo[i * n + c] = f[i * n + c];
            } else {
                int64_t s = pull_source(p, x, y, z, i, &bounced);
                fo[i * n + c] = f[(bounced ? OPP[i] : i) * n + s];
            }
        }
    }
}

/* Macroscopic fields of the stored populations: out = [rho, ux, uy, uz, T]
 * (each N, NaN at solid cells; Neumann cells report the cell they copy).
 * totals = [mass, momentum x, y, z, total energy sum (f|xi|^2 + g)/2] over
 * fluid cells. */
void orc_moments(const orc_params *p, const double *f, const double *g, double *out, double *totals)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    int64_t c;
    double tm = 0.0, tx = 0.0, ty = 0.0, tz = 0.0, te = 0.0;
    make_tables();
    for (c = 0; c < n; ++c) {
        int x = (int)(c % p->nx);
        int y = (int)((c / p->nx) % p->ny);
        int z = (int)(c / ((int64_t)p->nx * p->ny));
        int t = cell_type(p, x, y, z);
        int64_t s = c;
        double fi[NQ], gi[NQ], rho, u[3], T;
        int i;
        if (t == CELL_SOLID) {
            for (i = 0; i < 5; ++i) out[i * n + c] = NAN;
            continue;
        }
        if (t == CELL_NEUMANN) s = neumann_source(p, x, y, z);
        for (i = 0; i < NQ; ++i) {
            fi[i] = f[i * n + s];
            gi[i] = g[i * n + s];
        }
        macroscopic(fi, gi, p->gamma, &rho, u, &T);
        out[c] = rho;
        out[n + c] = u[0];
        out[2 * n + c] = u[1];
        out[3 * n + c] = u[2];
        out[4 * n + c] = T;
        if (t == CELL_FLUID) {
            double e = 0.0;
            for (i = 0; i < NQ; ++i)
                e += fi[i] * (VEL[i][0] * VEL[i][0] + VEL[i][1] * VEL[i][1] + VEL[i][2] * VEL[i][2]) + gi[i];
            tm += rho;
            tx += rho * u[0];
            ty += rho * u[1];
            tz += rho * u[2];
            te += 0.5 * e;
        }
    }
    if (totals) {
        totals[0] = tm;
        totals[1] = tx;
        totals[2] = ty;
        totals[3] = tz;
        totals[4] = te;
    }
}
