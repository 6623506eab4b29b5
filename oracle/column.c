/*
 * ORACLE (test infrastructure only): the semi-implicit vertical column solve
 * and the finite-volume pressure-gradient force.
 *
 * The paper describes riem_solver_c as solving for the nonhydrostatic terms
 * of vertical velocity and pressure perturbation with a tridiagonal solver
 * (Sec. IX-B, citing Chen et al.); it prints no equations.  The column solve
 * below is the backward-Euler (off-centring 1) treatment of vertically
 * propagating sound on Lagrangian layers, written from its mathematics:
 *
 *   hydrostatic interface pressure  pi_{K+1} = pi_K + dpi_k   (top down)
 *   layer mass m_k = dpi_k / g, thickness h_k = -delz_k
 *   nonhydrostatic pressure from the equation of state
 *        p_k = p0 (Rd theta_k m_k / (h_k p0))^gamma
 *   perturbation about the log-mean hydrostatic pressure, interpolated to
 *   interfaces with mass weights (0 at the top, the last layer's at the
 *   bottom); momentum m_k dw_k/dt = P'_{k+1} - P'_k with the interface
 *   pressure linearised implicitly in w:
 *        P_K^{n+1} = P*_K - gamma P*_K dt (w_{K-1} - w_K) / d_K,
 *   which gives a symmetric, strictly diagonally dominant tridiagonal system
 *   solved by Thomas elimination; the new perturbation follows by a top-down
 *   scan of m (w_new - w)/dt, the new thickness by inverting the equation of
 *   state, and heights by a bottom-up scan from the surface.
 *
 * Interface perturbation (order 4): at interfaces with two layers on each
 * side, the value there of the cubic (in the mass coordinate) whose means
 * over those four layers are their perturbations, in place of the
 * mass-weighted mean of the two adjacent layers (order 2).
 *
 * Off-centring (weight beta in [0.5, 1], 1 = backward Euler above): the
 * momentum equation sees P^b = beta P^{n+1} + (1 - beta) P* and the pressure
 * response is driven by w^b = beta w^{n+1} + (1 - beta) w^n.  Eliminating
 * P^{n+1} leaves the same tridiagonal form with the coupling scaled by
 * beta^2 and the explicit part (1 - beta)/beta times the coupling acting on
 * w^n on the right-hand side; the top-down scan of m (w_new - w)/dt then
 * gives P^b, and P^{n+1} = (P^b - (1 - beta) P*)/beta enters the equation of
 * state.
 *
 * The pressure-gradient force is the contour integral of p dPhi around the
 * quadrilateral spanned by two columns and two interfaces (Green's theorem),
 * divided by the mean layer mass and the distance between the columns.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>

/* Interface values of the layer perturbation pp (K = 0 .. nz): 0 at the top,
 * the bottom layer's value at the surface; between layers the mass-weighted
 * mean of the two adjacent layers (order 2), or (order 4, where two layers lie
 * on each side) the interface value of the cubic whose means over the layers
 * K-2 .. K+1 equal their pp: a 4 x 4 linear system for the cubic's
 * coefficients in x = (mass coordinate - interface) / (dpi[K-1] + dpi[K]),
 * solved by Gaussian elimination with partial pivoting. */
void o_pp_interfaces(int nz, int order, const double *dpi, const double *pp, double *pps)
{
    pps[0] = 0.0;
    pps[nz] = pp[nz - 1];
    for (int K = 1; K < nz; K++) {
        if (order != 4 || K < 2 || K > nz - 2) {
            pps[K] = (dpi[K] * pp[K - 1] + dpi[K - 1] * pp[K]) / (dpi[K - 1] + dpi[K]);
            continue;
        }
        double sc = dpi[K - 1] + dpi[K];
        double e[5];
        e[2] = 0.0;
        e[1] = -dpi[K - 1] / sc;
        e[0] = e[1] - dpi[K - 2] / sc;
        e[3] = dpi[K] / sc;
        e[4] = e[3] + dpi[K + 1] / sc;
        double M[4][5];
        for (int r = 0; r < 4; r++) {
            double a = e[r], b = e[r + 1];
            for (int q = 0; q < 4; q++) M[r][q] = (pow(b, q + 1) - pow(a, q + 1)) / ((q + 1) * (b - a));
            M[r][4] = pp[K - 2 + r];
        }
        for (int c = 0; c < 4; c++) {
            int piv = c;
            for (int r = c + 1; r < 4; r++)
                if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
            for (int q = 0; q < 5; q++) {
                double tmp = M[c][q];
                M[c][q] = M[piv][q];
                M[piv][q] = tmp;
            }
            for (int r = c + 1; r < 4; r++) {
                double f = M[r][c] / M[c][c];
                for (int q = c; q < 5; q++) M[r][q] -= f * M[c][q];
            }
        }
        double co[4];
        for (int c = 3; c >= 0; c--) {
            double v = M[c][4];
            for (int q = c + 1; q < 4; q++) v -= M[c][q] * co[q];
            co[c] = v / M[c][c];
        }
        pps[K] = co[0];   /* the cubic at x = 0 */
    }
}

/* Returns the smallest Thomas pivot (positive for a well-posed column). */
double o_sim1b(int nz, double dt, double beta, int pp_order, double ptop, double zs, const double *dpi,
               const double *theta, const double *delz, const double *w, double *w_out,
               double *delz_out, double *pfull, double *phi, double *pstar, double *coupling)
{
    const double g = O_GRAV, rd = O_RDGAS, kappa = O_RDGAS / O_CP;
    const double gam = 1.0 / (1.0 - kappa), p0 = O_P0;
    double *pi = (double *)malloc(sizeof(double) * (nz + 1));
    double *pibar = (double *)malloc(sizeof(double) * nz);
    double *m = (double *)malloc(sizeof(double) * nz);
    double *h = (double *)malloc(sizeof(double) * nz);
    double *pp = (double *)malloc(sizeof(double) * nz);
    double *pps = (double *)malloc(sizeof(double) * (nz + 1));
    double *A = (double *)malloc(sizeof(double) * (nz + 1));
    double *cp = (double *)malloc(sizeof(double) * nz);
    double *dp = (double *)malloc(sizeof(double) * nz);
    double *ppn = (double *)malloc(sizeof(double) * (nz + 1));
    double minpiv = 1e300;

    pi[0] = ptop;
    for (int k = 0; k < nz; k++) pi[k + 1] = pi[k] + dpi[k];
    for (int k = 0; k < nz; k++) {
        pibar[k] = dpi[k] / (log(pi[k + 1]) - log(pi[k]));
        m[k] = dpi[k] / g;
        h[k] = -delz[k];
        double p = p0 * pow(rd * theta[k] * m[k] / (h[k] * p0), gam);
        pp[k] = p - pibar[k];
    }
    o_pp_interfaces(nz, pp_order, dpi, pp, pps);
    /* coupling of interface K: dt times the linearised pressure response to
     * the convergence of w, times beta^2 (see the header) */
    A[0] = 0.0;
    for (int K = 1; K <= nz; K++) {
        double d = K < nz ? 0.5 * (h[K - 1] + h[K]) : 0.5 * h[nz - 1];
        A[K] = beta * beta * gam * (pi[K] + pps[K]) * dt * dt / d;
        if (coupling) coupling[K] = gam * (pi[K] + pps[K]) * dt / d;
    }
    if (coupling) coupling[0] = 0.0;
    if (pstar)
        for (int K = 0; K <= nz; K++) pstar[K] = pps[K];
    const double ex = (1.0 - beta) / beta;
    /* Thomas elimination: lower -A[k], diagonal m + A[k] + A[k+1], upper -A[k+1] */
    for (int k = 0; k < nz; k++) {
        double lower = k > 0 ? -A[k] : 0.0;
        double diag = m[k] + A[k] + A[k + 1];
        double upper = k < nz - 1 ? -A[k + 1] : 0.0;
        double rhs = m[k] * w[k] + dt * (pps[k + 1] - pps[k]);   /* surface w = 0 */
        if (beta != 1.0) {
            double wa = k > 0 ? w[k - 1] : 0.0, wb = k < nz - 1 ? w[k + 1] : 0.0;
            rhs -= ex * (A[k + 1] * (w[k] - wb) - A[k] * (wa - w[k]));
        }
        double piv = k > 0 ? diag - lower * cp[k - 1] : diag;
        if (piv < minpiv) minpiv = piv;
        cp[k] = upper / piv;
        dp[k] = (k > 0 ? rhs - lower * dp[k - 1] : rhs) / piv;
    }
    w_out[nz - 1] = dp[nz - 1];
    for (int k = nz - 2; k >= 0; k--) w_out[k] = dp[k] - cp[k] * w_out[k + 1];

    /* the scan gives the off-centred perturbation; the new one follows */
    ppn[0] = 0.0;
    for (int k = 0; k < nz; k++) ppn[k + 1] = ppn[k] + m[k] * (w_out[k] - w[k]) / dt;
    if (beta != 1.0)
        for (int K = 0; K <= nz; K++) ppn[K] = (ppn[K] - (1.0 - beta) * pps[K]) / beta;
    double z = zs;
    if (phi) phi[nz] = g * z;
    double *hn = (double *)malloc(sizeof(double) * nz);
    for (int k = 0; k < nz; k++) {
        double pn = pibar[k] + 0.5 * (ppn[k] + ppn[k + 1]);
        hn[k] = rd * theta[k] * m[k] / p0 * pow(p0 / pn, 1.0 / gam);
    }
    for (int k = nz - 1; k >= 0; k--) {
        z = z + hn[k];
        if (phi) phi[k] = g * z;
    }
    for (int k = 0; k < nz; k++) delz_out[k] = -hn[k];
    if (pfull)
        for (int K = 0; K <= nz; K++) pfull[K] = pi[K] + ppn[K];
    free(pi); free(pibar); free(m); free(h); free(pp); free(pps); free(A);
    free(cp); free(dp); free(ppn); free(hn);
    return minpiv;
}

double o_sim1(int nz, double dt, double ptop, double zs, const double *dpi, const double *theta,
              const double *delz, const double *w, double *w_out, double *delz_out,
              double *pfull, double *phi)
{
    return o_sim1b(nz, dt, 1.0, 2, ptop, zs, dpi, theta, delz, w, w_out, delz_out, pfull, phi, 0, 0);
}

double o_pgf(double dt, double L, double dpiW, double dpiE, double phW0, double phW1,
             double phE0, double phE1, double pW0, double pW1, double pE0, double pE1)
{
    return dt / (L * (dpiW + dpiE)) *
           ((phW1 - phE0) * (pE1 - pW0) + (phW0 - phE1) * (pW1 - pE0));
}
