/*
 * lbm_oracle.c -- plain, slow, single-threaded FP64 reference of MinxEnt-LBM
 * (T. L. Wilson, M. Pugh, F. Dawson, "Stabilization of the Lattice Boltzmann
 * Method Using Information Theory", arXiv:1801.03863).
 *
 * TEST INFRASTRUCTURE ONLY.  The HIP library never links, loads or calls this
 * file and shares no code, header, table or helper with it.  Only the test
 * suite, the package smoke check and the CPU-baseline leg of the benchmark use
 * it.  Every step follows the paper's order and notation; nothing is blocked,
 * fused or reordered for speed.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -std=c11 -shared -fPIC
 *
 * Conventions (readings of the paper, each listed with its reason in the
 * design notes of the repository):
 *  - D2Q9 populations are indexed in the column order of the moment matrix T
 *    of Sec. IV.D: rest, E, N, W, S, NE, NW, SW, SE.  Table I lists the same
 *    nine velocities and weights with the rest velocity last; T's second row
 *    puts -4 on the rest column and its fourth row is j_x, which fixes the
 *    order used here.
 *  - D1Q3 populations are (rest, +1, -1) with weights (2/3, 1/6, 1/6), the
 *    one-dimensional factor of Table I's weights.  With mass, momentum and the
 *    relaxed second moment as constraints no moment is left free (Sec. IV.F
 *    says D1Q3 is over-constrained), so the collision is exactly SRT.
 *  - Nodes whose Newton start point has a non-positive population cannot take
 *    the logarithm; they keep the start point (m1 = m0) and are counted as
 *    "guarded".  Values are never clipped.
 *  - A whole run is: initial populations at equilibrium (Sec. IV.E), then per
 *    time step a per-node role collision (fluid: the chosen collision rule;
 *    wall: full-way bounce-back; moving lid: equilibrium at the lid density
 *    and velocity, Sec. IV.E) followed by push streaming (Sec. II.A).  A slot
 *    whose upstream node lies outside the lattice keeps its old value; such
 *    slots only ever sit on boundary nodes and never reach a fluid node.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Lattice constants                                                         */
/* ------------------------------------------------------------------------ */

/* Table I velocities, permuted to the column order of T (Sec. IV.D). */
static const int VX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int VY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Table I weights in the same order. */
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* The moment matrix T exactly as printed in Sec. IV.D. */
static const double T[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

/* Full-way bounce-back partner of each direction (Sec. IV.E). */
static const int OPP9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* D1Q3: velocities (0, +1, -1), weights (2/3, 1/6, 1/6). */
static const int V3[3] = {0, 1, -1};
static const double W3[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
static const int OPP3[3] = {0, 2, 1};

/* T^{-1}, computed once by Gauss-Jordan elimination with partial pivoting in
 * long double and rounded to double.  No shortcut (such as the orthogonality
 * of T's rows) is used here; the tests check the result against one. */
static double TINV[9][9];
static int tinv_ready = 0;

static void ensure_tinv(void)
{
    if (tinv_ready) return;
    long double a[9][18];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 18; ++j)
            a[i][j] = (j < 9) ? (long double)T[i][j] : (long double)((j - 9) == i);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabsl(a[r][c]) > fabsl(a[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 18; ++j) {
                long double t = a[c][j];
                a[c][j] = a[piv][j];
                a[piv][j] = t;
            }
        long double d = a[c][c];
        for (int j = 0; j < 18; ++j) a[c][j] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == c) continue;
            long double m = a[r][c];
            if (m == 0.0L) continue;
            for (int j = 0; j < 18; ++j) a[r][j] -= m * a[c][j];
        }
    }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) TINV[i][j] = (double)a[i][j + 9];
    tinv_ready = 1;
}

/* ------------------------------------------------------------------------ */
/* Small exported helpers (the tests pin each of them)                       */
/* ------------------------------------------------------------------------ */

void orc_constants(double *t_out, double *tinv_out, double *w_out, int *vx_out, int *vy_out)
{
    ensure_tinv();
    for (int i = 0; i < 9; ++i) {
        for (int j = 0; j < 9; ++j) {
            if (t_out) t_out[9 * i + j] = T[i][j];
            if (tinv_out) tinv_out[9 * i + j] = TINV[i][j];
        }
        if (w_out) w_out[i] = W[i];
        if (vx_out) vx_out[i] = VX[i];
        if (vy_out) vy_out[i] = VY[i];
    }
}

/* Polynomial equilibrium, Sec. IV.E:
 * f_eq = W rho (1 + 3 v.u + 9/2 (v.u)^2 - 3/2 |u|^2). */
void orc_feq_d2q9(double rho, double ux, double uy, double *out)
{
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double cu = VX[a] * ux + VY[a] * uy;
        out[a] = W[a] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* The same equilibrium on the D1Q3 set. */
void orc_feq_d1q3(double rho, double ux, double *out)
{
    for (int a = 0; a < 3; ++a) {
        double cu = V3[a] * ux;
        out[a] = W3[a] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
    }
}

/* Discrete Kullback-Leibler divergence from the lattice weights,
 * H(p) = sum_a p_a ln(p_a / W_a)  (Sec. IV.B). */
double orc_kld_d2q9(const double *p)
{
    double h = 0.0;
    for (int a = 0; a < 9; ++a) h += p[a] * log(p[a] / W[a]);
    return h;
}

/* Gaussian elimination with partial pivoting for an n x n system (n <= 9).
 * a is row-major and overwritten; b is overwritten with the solution. */
static void gauss_solve(int n, double *a, double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * n + c]) > fabs(a[piv * n + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                double t = a[c * n + j];
                a[c * n + j] = a[piv * n + j];
                a[piv * n + j] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double m = a[r * n + c] / a[c * n + c];
            for (int j = c; j < n; ++j) a[r * n + j] -= m * a[c * n + j];
            b[r] -= m * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < n; ++j) s -= a[r * n + j] * b[j];
        b[r] = s / a[r * n + r];
    }
}

/* ------------------------------------------------------------------------ */
/* Collision rules                                                           */
/* ------------------------------------------------------------------------ */

/* Shared set-up of the MinxEnt problem for one node (Sec. IV.C and IV.D):
 * rho, u, the start moment vector M0 (equilibrium moments of the node's own
 * rho and u, with the constrained entries set to the constraint values) and
 * the list of free moment indices (0-based rows of T).  variant 4: free rows
 * {2,3,5,7} (1-based); variant 2: free rows {2,3}. */
static int minxent_setup(const double *f, double tau, double tau2, int variant,
                         double *rho_out, double *M0, int *free_idx)
{
    ensure_tinv();
    /* f = rho p, eq. for f and p in Sec. III.A. */
    double rho = 0.0;
    for (int a = 0; a < 9; ++a) rho += f[a];
    double p[9];
    for (int a = 0; a < 9; ++a) p[a] = f[a] / rho;
    /* u from the momentum constraints C4 and C6 (Sec. IV.C). */
    double ux = 0.0, uy = 0.0;
    for (int a = 0; a < 9; ++a) {
        ux += p[a] * VX[a];
        uy += p[a] * VY[a];
    }
    /* Equilibrium probabilities: the polynomial equilibrium divided by rho. */
    double peq[9];
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double cu = VX[a] * ux + VY[a] * uy;
        peq[a] = W[a] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
    /* Step 1 of the algorithm in Sec. IV.D: pre-collision and equilibrium
     * moments, then the constraint values. */
    double Mpre[9], Meq[9];
    for (int i = 0; i < 9; ++i) {
        Mpre[i] = 0.0;
        Meq[i] = 0.0;
        for (int a = 0; a < 9; ++a) {
            Mpre[i] += T[i][a] * p[a];
            Meq[i] += T[i][a] * peq[a];
        }
    }
    for (int i = 0; i < 9; ++i) M0[i] = Meq[i];
    M0[0] = 1.0; /* C1: sum p = 1 */
    M0[3] = ux;  /* C4 */
    M0[5] = uy;  /* C6 */
    /* C8 and C9: the stress moments relaxed by 1/tau toward equilibrium. */
    M0[7] = Mpre[7] + (Meq[7] - Mpre[7]) / tau;
    M0[8] = Mpre[8] + (Meq[8] - Mpre[8]) / tau;
    int nfree;
    if (variant == 2) {
        /* C5 and C7 (MinxEnt2): relaxed by 1/tau2. */
        M0[4] = Mpre[4] + (Meq[4] - Mpre[4]) / tau2;
        M0[6] = Mpre[6] + (Meq[6] - Mpre[6]) / tau2;
        free_idx[0] = 1;
        free_idx[1] = 2;
        nfree = 2;
    } else {
        free_idx[0] = 1;
        free_idx[1] = 2;
        free_idx[2] = 4;
        free_idx[3] = 6;
        nfree = 4;
    }
    *rho_out = rho;
    return nfree;
}

/* p = T^{-1} M. */
static void moments_to_p(const double *M, double *p)
{
    for (int a = 0; a < 9; ++a) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += TINV[a][i] * M[i];
        p[a] = s;
    }
}

/* Gradient and Hessian of S(M) = H(T^{-1} M) with respect to the free
 * moments (Sec. IV.D).  Returns 0 if some population is non-positive or not
 * finite, in which case the logarithm is undefined. */
static int grad_hess(const double *M, const int *free_idx, int nfree, double *g, double *H)
{
    double p[9];
    moments_to_p(M, p);
    for (int a = 0; a < 9; ++a)
        if (!(p[a] > 0.0) || !isfinite(p[a])) return 0;
    for (int k = 0; k < nfree; ++k) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += TINV[a][free_idx[k]] * (log(p[a] / W[a]) + 1.0);
        g[k] = s;
    }
    for (int j = 0; j < nfree; ++j)
        for (int k = 0; k < nfree; ++k) {
            double s = 0.0;
            for (int a = 0; a < 9; ++a)
                s += TINV[a][free_idx[k]] * TINV[a][free_idx[j]] / p[a];
            H[j * nfree + k] = s;
        }
    return 1;
}

/* MinxEnt collision with one Newton-Raphson step (Sec. IV.D, the five-step
 * algorithm).  variant 4 = MinxEnt4, 2 = MinxEnt2.  Writes f_post = rho p_post.
 * Returns 1 if the node was guarded (start point outside p > 0). */
int orc_collide_minxent(const double *f, double tau, double tau2, int variant, double *out)
{
    double rho, M0[9];
    int free_idx[4];
    int nfree = minxent_setup(f, tau, tau2, variant, &rho, M0, free_idx);
    /* Step 2: gradient and Hessian at the start point. */
    double g[4], H[16];
    double Mpost[9];
    for (int i = 0; i < 9; ++i) Mpost[i] = M0[i];
    int ok = grad_hess(M0, free_idx, nfree, g, H);
    if (ok) {
        /* Step 3: m1 = m0 - H^{-1} grad S; a single step. */
        gauss_solve(nfree, H, g);
        /* Step 4: full post-collision moment vector. */
        for (int k = 0; k < nfree; ++k) Mpost[free_idx[k]] = M0[free_idx[k]] - g[k];
    }
    /* Step 5: back to distribution space, then f = rho p. */
    double p[9];
    moments_to_p(Mpost, p);
    for (int a = 0; a < 9; ++a) out[a] = rho * p[a];
    return ok ? 0 : 1;
}

/* The Newton start point alone: p0 = T^{-1} M0 times rho (used by tests). */
void orc_minxent_start(const double *f, double tau, double tau2, int variant, double *out)
{
    double rho, M0[9], p[9];
    int free_idx[4];
    minxent_setup(f, tau, tau2, variant, &rho, M0, free_idx);
    moments_to_p(M0, p);
    for (int a = 0; a < 9; ++a) out[a] = rho * p[a];
}

/* The converged constrained minimiser, by damped Newton iteration over the
 * free moments in long double until the gradient is below tol (brute force,
 * used to pin the single step).  Returns the iteration count, or -1 if it did
 * not converge. */
int orc_converged_minxent(const double *f, double tau, double tau2, int variant,
                          int maxit, double tol, double *out)
{
    double rho, M0d[9];
    int free_idx[4];
    int nfree = minxent_setup(f, tau, tau2, variant, &rho, M0d, free_idx);
    long double M[9], ti[9][9], wl[9];
    for (int i = 0; i < 9; ++i) M[i] = M0d[i];
    for (int a = 0; a < 9; ++a) {
        wl[a] = (long double)W[a];
        for (int i = 0; i < 9; ++i) ti[a][i] = (long double)TINV[a][i];
    }
    int it;
    for (it = 0; it < maxit; ++it) {
        long double p[9], g[4], H[16];
        for (int a = 0; a < 9; ++a) {
            p[a] = 0.0L;
            for (int i = 0; i < 9; ++i) p[a] += ti[a][i] * M[i];
            if (!(p[a] > 0.0L)) return -1;
        }
        long double S0 = 0.0L;
        for (int a = 0; a < 9; ++a) S0 += p[a] * logl(p[a] / wl[a]);
        long double gmax = 0.0L;
        for (int k = 0; k < nfree; ++k) {
            g[k] = 0.0L;
            for (int a = 0; a < 9; ++a) g[k] += ti[a][free_idx[k]] * (logl(p[a] / wl[a]) + 1.0L);
            if (fabsl(g[k]) > gmax) gmax = fabsl(g[k]);
        }
        if (gmax < (long double)tol) break;
        for (int j = 0; j < nfree; ++j)
            for (int k = 0; k < nfree; ++k) {
                H[j * nfree + k] = 0.0L;
                for (int a = 0; a < 9; ++a)
                    H[j * nfree + k] += ti[a][free_idx[k]] * ti[a][free_idx[j]] / p[a];
            }
        /* Solve H d = g (Gaussian elimination, partial pivoting). */
        long double d[4];
        for (int k = 0; k < nfree; ++k) d[k] = g[k];
        for (int c = 0; c < nfree; ++c) {
            int piv = c;
            for (int r = c + 1; r < nfree; ++r)
                if (fabsl(H[r * nfree + c]) > fabsl(H[piv * nfree + c])) piv = r;
            if (piv != c) {
                for (int j = 0; j < nfree; ++j) {
                    long double t = H[c * nfree + j];
                    H[c * nfree + j] = H[piv * nfree + j];
                    H[piv * nfree + j] = t;
                }
                long double t = d[c];
                d[c] = d[piv];
                d[piv] = t;
            }
            for (int r = c + 1; r < nfree; ++r) {
                long double m = H[r * nfree + c] / H[c * nfree + c];
                for (int j = c; j < nfree; ++j) H[r * nfree + j] -= m * H[c * nfree + j];
                d[r] -= m * d[c];
            }
        }
        for (int r = nfree - 1; r >= 0; --r) {
            long double s = d[r];
            for (int j = r + 1; j < nfree; ++j) s -= H[r * nfree + j] * d[j];
            d[r] = s / H[r * nfree + r];
        }
        /* Damping: halve the step until every population stays positive and
         * the divergence does not increase. */
        long double step = 1.0L;
        for (int tries = 0; tries < 60; ++tries) {
            long double Mt[9], pt[9], St = 0.0L;
            int pos = 1;
            for (int i = 0; i < 9; ++i) Mt[i] = M[i];
            for (int k = 0; k < nfree; ++k) Mt[free_idx[k]] -= step * d[k];
            for (int a = 0; a < 9 && pos; ++a) {
                pt[a] = 0.0L;
                for (int i = 0; i < 9; ++i) pt[a] += ti[a][i] * Mt[i];
                if (!(pt[a] > 0.0L)) pos = 0;
            }
            if (pos) {
                for (int a = 0; a < 9; ++a) St += pt[a] * logl(pt[a] / wl[a]);
                if (St <= S0 + 1e-18L) {
                    for (int i = 0; i < 9; ++i) M[i] = Mt[i];
                    break;
                }
            }
            step *= 0.5L;
        }
    }
    if (it >= maxit) return -1;
    for (int a = 0; a < 9; ++a) {
        long double s = 0.0L;
        for (int i = 0; i < 9; ++i) s += ti[a][i] * M[i];
        out[a] = (double)((long double)rho * s);
    }
    return it;
}

/* SRT / lattice BGK, Sec. II.B.1: f + (f_eq - f) / tau. */
void orc_collide_srt_d2q9(const double *f, double tau, double *out)
{
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        rho += f[a];
        jx += f[a] * VX[a];
        jy += f[a] * VY[a];
    }
    double feq[9];
    orc_feq_d2q9(rho, jx / rho, jy / rho, feq);
    for (int a = 0; a < 9; ++a) out[a] = f[a] + (feq[a] - f[a]) / tau;
}

/* MRT, Sec. II.B.2: f + T^{-1} B T (f_eq - f) with B = diag(b); Table III
 * gives b for MRT, TRT and SRT. */
void orc_collide_mrt_d2q9(const double *f, const double *b, double *out)
{
    ensure_tinv();
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        rho += f[a];
        jx += f[a] * VX[a];
        jy += f[a] * VY[a];
    }
    double feq[9], d[9], m[9];
    orc_feq_d2q9(rho, jx / rho, jy / rho, feq);
    for (int a = 0; a < 9; ++a) d[a] = feq[a] - f[a];
    for (int i = 0; i < 9; ++i) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += T[i][a] * d[a];
        m[i] = b[i] * s;
    }
    for (int a = 0; a < 9; ++a) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += TINV[a][i] * m[i];
        out[a] = f[a] + s;
    }
}

/* D1Q3 SRT: f + (f_eq - f) / tau. */
void orc_collide_srt_d1q3(const double *f, double tau, double *out)
{
    double rho = f[0] + f[1] + f[2];
    double ux = (f[1] - f[2]) / rho;
    double feq[3];
    orc_feq_d1q3(rho, ux, feq);
    for (int a = 0; a < 3; ++a) out[a] = f[a] + (feq[a] - f[a]) / tau;
}

/* D1Q3 in moment form with no free moment: M = T1 f with rows (1, v, v^2);
 * mass and momentum kept, the second moment relaxed by 1/tau toward its
 * equilibrium value, and f = T1^{-1} M. */
void orc_collide_moment_d1q3(const double *f, double tau, double *out)
{
    double M0 = f[0] + f[1] + f[2];
    double M1 = f[1] - f[2];
    double M2 = f[1] + f[2];
    double feq[3];
    orc_feq_d1q3(M0, M1 / M0, feq);
    double M2eq = feq[1] + feq[2];
    double M2post = M2 + (M2eq - M2) / tau;
    /* T1^{-1}: f_rest = M0 - M2, f_+ = (M2 + M1)/2, f_- = (M2 - M1)/2. */
    out[0] = M0 - M2post;
    out[1] = 0.5 * (M2post + M1);
    out[2] = 0.5 * (M2post - M1);
}

/* ------------------------------------------------------------------------ */
/* Whole runs                                                                */
/* ------------------------------------------------------------------------ */

enum { ORC_D1Q3 = 1, ORC_D2Q9 = 2 };
enum { ORC_MINXENT4 = 0, ORC_MINXENT2 = 1, ORC_SRT = 2, ORC_TRT = 3, ORC_MRT = 4, ORC_CONVERGED4 = 5 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_TUBE = 1, ORC_BC_CAVITY = 2, ORC_BC_BOX = 3 };
enum { ROLE_FLUID = 0, ROLE_WALL = 1, ROLE_LID = 2 };

typedef struct {
    int32_t lattice, collision, bc, pad;
    int32_t nx, ny;
    double tau, tau2, u_lid, rho0;
} orc_params;

typedef struct {
    int32_t unstable;   /* 1 if some fluid post-collision population was negative or not finite */
    int32_t first_step; /* step of the first such event, -1 if none */
    int64_t guarded;    /* node-steps where the Newton start point left p > 0 */
    int64_t first_node; /* smallest node index x + y*nx (whole lattice) unstable at first_step, -1 if none */
    double min_post;    /* smallest fluid post-collision population over the steps up to and including
                           first_step (the whole run if stable); -inf for a non-finite one.  A record of
                           how close a run came to the stability criterion of Sec. IV.G, not part of it. */
} orc_status;

/* Node role from its global coordinates.  Tube: walls at x = 0 and x = nx-1
 * (y is periodic).  Cavity: the top row y = ny-1 (corners included) is the
 * lid; x = 0, x = nx-1 and y = 0 are walls.  Box: walls on all four sides. */
static int node_role(const orc_params *P, int x, int y)
{
    int nx = P->nx, ny = P->ny;
    switch (P->bc) {
    case ORC_BC_TUBE:
        return (x == 0 || x == nx - 1) ? ROLE_WALL : ROLE_FLUID;
    case ORC_BC_CAVITY:
        if (P->lattice == ORC_D2Q9 && y == ny - 1) return ROLE_LID;
        if (x == 0 || x == nx - 1) return ROLE_WALL;
        if (P->lattice == ORC_D2Q9 && y == 0) return ROLE_WALL;
        return ROLE_FLUID;
    case ORC_BC_BOX:
        if (x == 0 || x == nx - 1) return ROLE_WALL;
        if (P->lattice == ORC_D2Q9 && (y == 0 || y == ny - 1)) return ROLE_WALL;
        return ROLE_FLUID;
    default:
        return ROLE_FLUID;
    }
}

static int x_periodic(const orc_params *P) { return P->bc == ORC_BC_PERIODIC; }
static int y_periodic(const orc_params *P) { return P->bc == ORC_BC_PERIODIC || P->bc == ORC_BC_TUBE; }

static void fluid_collide(const orc_params *P, const double *f, double *out, orc_status *st)
{
    if (P->lattice == ORC_D1Q3) {
        orc_collide_srt_d1q3(f, P->tau, out);
        return;
    }
    double b[9];
    switch (P->collision) {
    case ORC_MINXENT4:
        st->guarded += orc_collide_minxent(f, P->tau, P->tau2, 4, out);
        break;
    case ORC_MINXENT2:
        st->guarded += orc_collide_minxent(f, P->tau, P->tau2, 2, out);
        break;
    case ORC_SRT:
        orc_collide_srt_d2q9(f, P->tau, out);
        break;
    case ORC_TRT:
        /* Table III, TRT row. */
        b[0] = 0; b[1] = 1 / P->tau; b[2] = 1 / P->tau; b[3] = 0; b[4] = 1 / P->tau2;
        b[5] = 0; b[6] = 1 / P->tau2; b[7] = 1 / P->tau; b[8] = 1 / P->tau;
        orc_collide_mrt_d2q9(f, b, out);
        break;
    case ORC_MRT:
        /* Table III, MRT row. */
        b[0] = 0; b[1] = 1.64; b[2] = 1.54; b[3] = 0; b[4] = 1 / P->tau2;
        b[5] = 0; b[6] = 1 / P->tau2; b[7] = 1 / P->tau; b[8] = 1 / P->tau;
        orc_collide_mrt_d2q9(f, b, out);
        break;
    case ORC_CONVERGED4:
        if (orc_converged_minxent(f, P->tau, P->tau2, 4, 200, 1e-15, out) < 0)
            st->guarded += orc_collide_minxent(f, P->tau, P->tau2, 4, out);
        break;
    }
}

/* The fluid collision a whole run applies at one node under P (lattice,
 * collision rule, tau, tau2), exposed so that the tests can pin each rule's
 * relaxation rates (Table III) without a run.  b = 9 (D2Q9) or 3 (D1Q3)
 * populations in and out.  Returns 1 if the MinxEnt start point was guarded,
 * else 0. */
int orc_collide_node(const orc_params *P, const double *f, double *out)
{
    orc_status st = {0, -1, 0, -1, 0.0};
    fluid_collide(P, f, out, &st);
    return st.guarded != 0;
}

/* Run `steps` time steps on the window [x0, x0+wx) x [y0, y0+wy) of the
 * nx x ny lattice described by P, starting from the equilibrium of the given
 * fields (arrays of wx*wy values, x fastest; uy ignored for D1Q3).  Node roles
 * come from global coordinates.  An axis wraps only if it is periodic and the
 * window spans it; across the other window edges nothing streams in, so after
 * k steps only nodes at least k nodes away from such an edge are exact.
 * Writes rho and u of the final state into the *_out arrays (any may be NULL)
 * and, if f_out is not NULL, the final populations as b planes of wx*wy
 * values.  Returns 0, or -1 on bad parameters or allocation failure. */
int orc_run_window(const orc_params *P, int x0, int y0, int wx, int wy,
                   const double *rho_in, const double *ux_in, const double *uy_in,
                   int64_t steps, double *rho_out, double *ux_out, double *uy_out,
                   double *f_out, orc_status *st)
{
    const int b = (P->lattice == ORC_D1Q3) ? 3 : 9;
    const int gny = (P->lattice == ORC_D1Q3) ? 1 : P->ny;
    if (P->lattice == ORC_D1Q3) { y0 = 0; wy = 1; }
    if (P->nx < 3 || gny < 1 || !(P->tau > 0.5)) return -1;
    if (x0 < 0 || y0 < 0 || wx < 1 || wy < 1 || x0 + wx > P->nx || y0 + wy > gny) return -1;
    const int xwrap = x_periodic(P) && wx == P->nx;
    const int ywrap = y_periodic(P) && wy == gny;
    const size_t n = (size_t)wx * (size_t)wy;
    double *f = malloc(sizeof(double) * b * n);
    double *fp = malloc(sizeof(double) * b * n);
    unsigned char *role = malloc(n);
    if (!f || !fp || !role) {
        free(f);
        free(fp);
        free(role);
        return -1;
    }
    st->unstable = 0;
    st->first_step = -1;
    st->first_node = -1;
    st->guarded = 0;
    st->min_post = INFINITY;
    double flid[9];
    orc_feq_d2q9(P->rho0, P->u_lid, 0.0, flid);

    /* Initial state: equilibrium of the given fields (Sec. IV.E); the lid
     * starts at the equilibrium of the lid density and velocity. */
    for (int y = 0; y < wy; ++y)
        for (int x = 0; x < wx; ++x) {
            size_t i = (size_t)y * wx + x;
            role[i] = (unsigned char)node_role(P, x0 + x, y0 + y);
            double loc[9];
            if (b == 3) {
                orc_feq_d1q3(rho_in[i], ux_in[i], loc);
            } else if (role[i] == ROLE_LID) {
                for (int a = 0; a < 9; ++a) loc[a] = flid[a];
            } else {
                orc_feq_d2q9(rho_in[i], ux_in[i], uy_in[i], loc);
            }
            for (int a = 0; a < b; ++a) f[a * n + i] = loc[a];
        }

    for (int64_t s = 0; s < steps; ++s) {
        /* Collision by role. */
        for (size_t i = 0; i < n; ++i) {
            double loc[9], out[9];
            for (int a = 0; a < b; ++a) loc[a] = f[a * n + i];
            if (role[i] == ROLE_FLUID) {
                fluid_collide(P, loc, out, st);
                if (!st->unstable || st->first_step == (int32_t)s)
                    for (int a = 0; a < b; ++a) {
                        double v = isfinite(out[a]) ? out[a] : -INFINITY;
                        if (v < st->min_post) st->min_post = v;
                    }
                for (int a = 0; a < b; ++a)
                    if (!(out[a] >= 0.0) || !isfinite(out[a])) {
                        /* nodes are visited in increasing index, so the first one
                         * found in the first unstable step is the smallest */
                        if (!st->unstable) {
                            st->first_step = (int32_t)s;
                            st->first_node = (int64_t)(y0 + (int)(i / (size_t)wx)) * P->nx + (x0 + (int)(i % (size_t)wx));
                        }
                        st->unstable = 1;
                    }
            } else if (role[i] == ROLE_WALL) {
                for (int a = 0; a < b; ++a) out[a] = loc[(b == 3) ? OPP3[a] : OPP9[a]];
            } else {
                for (int a = 0; a < 9; ++a) out[a] = flid[a];
            }
            for (int a = 0; a < b; ++a) fp[a * n + i] = out[a];
        }
        /* Push streaming, Sec. II.A: f_a(x + v_a) <- post-collision f_a(x). */
        for (int a = 0; a < b; ++a) {
            int cx = (b == 3) ? V3[a] : VX[a];
            int cy = (b == 3) ? 0 : VY[a];
            for (int y = 0; y < wy; ++y)
                for (int x = 0; x < wx; ++x) {
                    int xd = x + cx, yd = y + cy;
                    if (xd < 0 || xd >= wx) {
                        if (!xwrap) continue;
                        xd = (xd + wx) % wx;
                    }
                    if (yd < 0 || yd >= wy) {
                        if (!ywrap) continue;
                        yd = (yd + wy) % wy;
                    }
                    f[a * n + (size_t)yd * wx + xd] = fp[a * n + (size_t)y * wx + x];
                }
        }
    }

    /* Macroscopic fields of the final state, Sec. II.A. */
    for (size_t i = 0; i < n; ++i) {
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int a = 0; a < b; ++a) {
            double v = f[a * n + i];
            rho += v;
            jx += v * ((b == 3) ? V3[a] : VX[a]);
            jy += v * ((b == 3) ? 0 : VY[a]);
        }
        if (rho_out) rho_out[i] = rho;
        if (ux_out) ux_out[i] = jx / rho;
        if (uy_out) uy_out[i] = jy / rho;
    }
    if (f_out) memcpy(f_out, f, sizeof(double) * b * n);
    free(f);
    free(fp);
    free(role);
    return 0;
}

/* The whole lattice. */
int orc_run(const orc_params *P, const double *rho_in, const double *ux_in, const double *uy_in,
            int64_t steps, double *rho_out, double *ux_out, double *uy_out, double *f_out,
            orc_status *st)
{
    int ny = (P->lattice == ORC_D1Q3) ? 1 : P->ny;
    return orc_run_window(P, 0, 0, P->nx, ny, rho_in, ux_in, uy_in, steps, rho_out, ux_out,
                          uy_out, f_out, st);
}
