/*
 * ORACLE (test infrastructure only): vertical remapping of the deformed
 * Lagrangian layers back to the reference ("Eulerian") coordinate.
 *
 * The paper places this step in the remapping timestep, after the tracer
 * advection and around the acoustic substeps (Sec. II; its cost is tuned
 * under "Lagrangian contrib." in Table III), and prints no equations.  The
 * readings taken here:
 *
 *  - Reference interfaces of a column: pe2_K = ak_K + bk_K ps (K = 0..nz),
 *    ps = ptop + sum of the column's delp, with ak_0 = ptop, bk_0 = 0,
 *    ak_nz = 0, bk_nz = 1, so that both ends of the column stay fixed and the
 *    column's mass is unchanged.
 *  - Each field is reconstructed in every source layer as a parabola in
 *    pressure (the piecewise-parabolic method of Colella and Woodward 1984 on
 *    non-uniform cells): interface values by the fourth-order interpolation
 *    of the layer means with monotonised slopes at interfaces that have two
 *    layers on each side, the thickness-weighted linear interpolation at the
 *    interfaces next to the top and bottom layers, constant top and bottom
 *    layers, then the monotonicity limiter on each parabola.
 *  - The new layer mean is the integral of the reconstruction over the
 *    reference layer divided by its thickness, which conserves the
 *    mass-weighted column integral exactly (up to rounding).
 *  - Fields: pt, w and the tracers are remapped as they are; delz as the
 *    ratio delz/delp, multiplied back by the new thickness (which keeps the
 *    column depth); the D-grid winds at faces, with the source and target
 *    interface pressures the mean of those of the two cells that share the
 *    face; delp becomes the reference thickness.
 *
 * Everything is FP64, one column at a time, with the overlap of every
 * source and target layer pair computed directly (no sweep).
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>

/* slope of layer j from the means of layers j-1, j, j+1 on thicknesses d,
 * monotonised: zero at a local extremum, else at most twice either one-sided
 * difference */
static double mono_slope(const double *d, const double *a, int j)
{
    double dm = a[j] - a[j - 1], dp = a[j + 1] - a[j];
    if (dm * dp <= 0.0) return 0.0;
    double s = d[j] / (d[j - 1] + d[j] + d[j + 1]) *
               ((2.0 * d[j - 1] + d[j]) / (d[j + 1] + d[j]) * dp + (d[j] + 2.0 * d[j + 1]) / (d[j - 1] + d[j]) * dm);
    double m = fabs(s);
    if (2.0 * fabs(dm) < m) m = 2.0 * fabs(dm);
    if (2.0 * fabs(dp) < m) m = 2.0 * fabs(dp);
    return s > 0.0 ? m : -m;
}

/* value at the interface between layers j and j+1 (needs j-1 and j+2) */
static double edge4(const double *d, const double *a, int j)
{
    double d0 = d[j - 1], d1 = d[j], d2 = d[j + 1], d3 = d[j + 2];
    double da = a[j + 1] - a[j];
    double v = a[j] + d1 / (d1 + d2) * da;
    double c = 2.0 * d2 * d1 / (d1 + d2) * ((d0 + d1) / (2.0 * d1 + d2) - (d3 + d2) / (2.0 * d2 + d1)) * da -
               d1 * (d0 + d1) / (2.0 * d1 + d2) * mono_slope(d, a, j + 1) +
               d2 * (d2 + d3) / (d1 + 2.0 * d2) * mono_slope(d, a, j);
    return v + c / (d0 + d1 + d2 + d3);
}

/* Interface values before the parabola limiter: e[K] (K = 1..nz-1) lies
 * between layers K-1 and K.  Exposed for tests. */
void o_ppm_edges(int nz, const double *d, const double *a, double *e)
{
    for (int K = 1; K < nz; K++) {
        if (K >= 2 && K <= nz - 2)
            e[K] = edge4(d, a, K - 1);
        else   /* next to the top or bottom layer: linear in pressure */
            e[K] = (a[K - 1] * d[K] + a[K] * d[K - 1]) / (d[K - 1] + d[K]);
    }
}

/* Parabola of every layer: left (top) value aL, right (bottom) value aR and
 * curvature a6, with q(x) = aL + x (aR - aL + a6 (1 - x)) for x in [0, 1]
 * from the top of the layer.  Exposed for tests. */
void o_ppm_profile(int nz, const double *d, const double *a, double *aL, double *aR, double *a6)
{
    double *e = (double *)malloc(sizeof(double) * (nz + 1));
    o_ppm_edges(nz, d, a, e);
    for (int k = 0; k < nz; k++) {
        double l, r, q = a[k];
        if (k == 0 || k == nz - 1) {
            l = r = q;
        } else {
            l = e[k];
            r = e[k + 1];
            /* monotonicity: flat at a local extremum, else move the edge that
             * puts the parabola's turning point inside the layer */
            if ((r - q) * (q - l) <= 0.0) {
                l = r = q;
            } else {
                double dq = r - l, c6 = 6.0 * (q - 0.5 * (l + r));
                if (dq * c6 > dq * dq)
                    l = 3.0 * q - 2.0 * r;
                else if (-dq * dq > dq * c6)
                    r = 3.0 * q - 2.0 * l;
            }
        }
        aL[k] = l;
        aR[k] = r;
        a6[k] = 6.0 * (q - 0.5 * (l + r));
    }
    free(e);
}

/* integral of the layer's parabola over x in [x1, x2] (fraction of the layer) */
static double parab_int(double l, double r, double c6, double x1, double x2)
{
    double s1 = x2 - x1, s2 = (x2 * x2 - x1 * x1) / 2.0, s3 = (x2 * x2 * x2 - x1 * x1 * x1) / 3.0;
    return l * s1 + (r - l) * s2 + c6 * (s2 - s3);
}

/* Remap one column: source interfaces pe1[0..nz], layer means q1, target
 * interfaces pe2[0..nz] (same end points) -> target means q2. */
void o_remap_column(int nz, const double *pe1, const double *pe2, const double *q1, double *q2)
{
    double *d = (double *)malloc(sizeof(double) * nz);
    double *aL = (double *)malloc(sizeof(double) * nz);
    double *aR = (double *)malloc(sizeof(double) * nz);
    double *a6 = (double *)malloc(sizeof(double) * nz);
    for (int k = 0; k < nz; k++) d[k] = pe1[k + 1] - pe1[k];
    o_ppm_profile(nz, d, q1, aL, aR, a6);
    for (int m = 0; m < nz; m++) {
        double top = pe2[m], bot = pe2[m + 1], mass = 0.0;
        for (int s = 0; s < nz; s++) {
            double lo = pe1[s] > top ? pe1[s] : top;
            double hi = pe1[s + 1] < bot ? pe1[s + 1] : bot;
            if (hi <= lo) continue;
            double x1 = (lo - pe1[s]) / d[s], x2 = (hi - pe1[s]) / d[s];
            mass += parab_int(aL[s], aR[s], a6[s], x1, x2) * d[s];
        }
        q2[m] = mass / (bot - top);
    }
    free(d);
    free(aL);
    free(aR);
    free(a6);
}

/* interfaces of a column from its thicknesses */
static void interfaces(int nz, double ptop, const double *dp, double *pe)
{
    pe[0] = ptop;
    for (int k = 0; k < nz; k++) pe[k + 1] = pe[k] + dp[k];
}

static void reference(int nz, const double *ak, const double *bk, double ps, double *pe)
{
    for (int K = 0; K <= nz; K++) pe[K] = ak[K] + bk[K] * ps;
}

/*
 * Remap a whole state in place (oracle layout f[t][k][j+3][i+3]).  The halo
 * of delp is filled first (the winds at tile-edge faces need the pressures
 * of the neighbouring tile's cells); q[0..nq) are cell fields.
 */
int orc_remap_impl(const OGrid *g, double *u, double *v, double *w, double *delp, double *pt,
                   double *delz, double *const *q, int nq, const double *ak, const double *bk)
{
    const int n = g->n, nz = g->nz;
    const size_t P = o_plane(g), L = (size_t)nz * P;
    og_fill_scalar(g, delp, nz, ST_C, 0);
    double *pe1 = (double *)malloc(sizeof(double) * (nz + 1));
    double *pe2 = (double *)malloc(sizeof(double) * (nz + 1));
    double *pa = (double *)malloc(sizeof(double) * (nz + 1));
    double *pb = (double *)malloc(sizeof(double) * (nz + 1));
    double *col = (double *)malloc(sizeof(double) * nz);
    double *out = (double *)malloc(sizeof(double) * nz);
    double *dp = (double *)malloc(sizeof(double) * nz);
    double *newdp = (double *)calloc(L * g->T, sizeof(double));

    for (int t = 0; t < g->T; t++) {
        const size_t o = (size_t)t * L;
        /* winds at faces first: they read the old thicknesses of two cells */
        for (int f = 0; f < 2; f++) {
            double *U = f == 0 ? u : v;
            int ni = f == 0 ? n : n + 1, nj = f == 0 ? n + 1 : n;
            int di = f == 0 ? 0 : -1, dj = f == 0 ? -1 : 0;   /* the other cell of the face */
            for (int j = 0; j < nj; j++)
                for (int i = 0; i < ni; i++) {
                    for (int k = 0; k < nz; k++) dp[k] = delp[o + k * P + IX(g, i, j)];
                    interfaces(nz, g->ptop, dp, pa);
                    for (int k = 0; k < nz; k++) dp[k] = delp[o + k * P + IX(g, i + di, j + dj)];
                    interfaces(nz, g->ptop, dp, pb);
                    for (int K = 0; K <= nz; K++) pe1[K] = 0.5 * (pa[K] + pb[K]);
                    reference(nz, ak, bk, 0.5 * (pa[nz] + pb[nz]), pe2);
                    for (int k = 0; k < nz; k++) col[k] = U[o + k * P + IX(g, i, j)];
                    o_remap_column(nz, pe1, pe2, col, out);
                    for (int k = 0; k < nz; k++) U[o + k * P + IX(g, i, j)] = out[k];
                }
        }
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                for (int k = 0; k < nz; k++) dp[k] = delp[o + k * P + IX(g, i, j)];
                interfaces(nz, g->ptop, dp, pe1);
                reference(nz, ak, bk, pe1[nz], pe2);
                double *F[3] = {pt, w, delz};
                for (int f = 0; f < 3 + nq; f++) {
                    double *X = f < 3 ? F[f] : q[f - 3];
                    for (int k = 0; k < nz; k++) {
                        col[k] = X[o + k * P + IX(g, i, j)];
                        if (f == 2) col[k] /= dp[k];   /* delz per unit pressure thickness */
                    }
                    o_remap_column(nz, pe1, pe2, col, out);
                    for (int k = 0; k < nz; k++)
                        X[o + k * P + IX(g, i, j)] = f == 2 ? out[k] * (pe2[k + 1] - pe2[k]) : out[k];
                }
                for (int k = 0; k < nz; k++) newdp[o + k * P + IX(g, i, j)] = pe2[k + 1] - pe2[k];
            }
    }
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    size_t x = (size_t)t * L + k * P + IX(g, i, j);
                    delp[x] = newdp[x];
                }
    free(pe1);
    free(pe2);
    free(pa);
    free(pb);
    free(col);
    free(out);
    free(dp);
    free(newdp);
    return 0;
}
