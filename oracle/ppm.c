/*
 * ORACLE (test infrastructure only): piecewise-parabolic face values and the
 * two-dimensional flux-form transport operator fv_tp_2d.
 *
 * fv_tp_2d computes fluxes for horizontal finite-volume transport; it is two
 * dimensional, mass conserving and works on one level at a time (Sec. IX-C,
 * citing the Lin & Rood multidimensional flux-form scheme).  The paper prints
 * no formula, so the operator below is the published Lin-Rood construction
 * written from its mathematics: an inner advective half update in each
 * direction, the outer 1-D PPM flux of the cross-updated field, and the
 * average of the two orderings.  The 1-D operator is a monotone PPM: a
 * limited slope per cell, fourth-order edge values, edge deviations clipped
 * to twice the slope, and the mean of the cell parabola over the swept
 * interval.  The unlimited order (hord 6, a reading of the "un-limited" PPM
 * option) keeps the fourth-order edges and the parabola but drops both
 * constraints: slopes (q+ - q-)/4 as they are, edge deviations unclipped.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double sgn(double x) { return x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0); }
static double min2(double a, double b) { return a < b ? a : b; }
static double max2(double a, double b) { return a > b ? a : b; }

/* limited slope of cell s from its two neighbours (zero at a local extremum) */
static double limited_slope(double qm, double q0, double qp)
{
    double d = (qp - qm) / 4.0;
    double qmax = max2(qm, max2(q0, qp)), qmin = min2(qm, min2(q0, qp));
    return sgn(d) * min2(fabs(d), min2(qmax - q0, q0 - qmin));
}

/* Face value between cells m-1 and m for Courant number c; q[0..5] holds the
 * cells m-3 .. m+2 along the sweep.  lim = 0: the unlimited order. */
double o_ppm_face_order(const double q[6], double c, int lim)
{
    double dm[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 1; s <= 4; s++)
        dm[s] = lim ? limited_slope(q[s - 1], q[s], q[s + 1]) : (q[s + 1] - q[s - 1]) / 4.0;
    /* left-edge value of cell s (s = 2, 3, 4 are m-1, m, m+1) */
    double al[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 2; s <= 4; s++) al[s] = 0.5 * (q[s - 1] + q[s]) + (dm[s - 1] - dm[s]) / 3.0;
    int s = c > 0.0 ? 2 : 3;
    double bl, br;
    if (lim) {
        bl = -sgn(dm[s]) * min2(2.0 * fabs(dm[s]), fabs(al[s] - q[s]));
        br = sgn(dm[s]) * min2(2.0 * fabs(dm[s]), fabs(al[s + 1] - q[s]));
    } else {
        bl = al[s] - q[s];
        br = al[s + 1] - q[s];
    }
    if (c > 0.0) return q[s] + (1.0 - c) * (br - c * (bl + br));
    return q[s] + (1.0 + c) * (bl + c * (bl + br));
}

double o_ppm_face(const double q[6], double c) { return o_ppm_face_order(q, c, 1); }

static double ppm_x(const OGrid *g, const double *q, int i, int j, double c)
{
    double a[6];
    for (int s = 0; s < 6; s++) a[s] = q[IX(g, i - 3 + s, j)];
    return o_ppm_face_order(a, c, g->hord != 6);
}
static double ppm_y(const OGrid *g, const double *q, int i, int j, double c)
{
    double a[6];
    for (int s = 0; s < 6; s++) a[s] = q[IX(g, i, j - 3 + s)];
    return o_ppm_face_order(a, c, g->hord != 6);
}

/*
 * One level of one tile.  q is the cell field (interior plus edge halos), qx
 * and qy its x-sweep and y-sweep corner views.  crx/xfx live on x-faces for
 * rows -3..n+2, cry/yfx on y-faces for columns -3..n+2.  Outputs FX on the
 * interior x-faces, FY on the interior y-faces, weighted by mx/my when given
 * (mass fluxes), else by the area fluxes.
 */
void o_fv_tp_2d(const OGrid *g, int t, const double *q, const double *qx, const double *qy,
                const double *crx, const double *cry, const double *xfx, const double *yfx,
                const double *mx, const double *my, double *FX, double *FY)
{
    int n = g->n;
    size_t P = o_plane(g);
    const double *area = g->area + (size_t)t * P;
    double *fy2 = (double *)calloc(P, sizeof(double));
    double *fx2 = (double *)calloc(P, sizeof(double));
    double *qi = (double *)calloc(P, sizeof(double));
    double *qj = (double *)calloc(P, sizeof(double));

    /* y-direction outer fluxes of q, and the inner advective y update */
    for (int j = 0; j <= n; j++)
        for (int i = -3; i <= n + 2; i++) fy2[IX(g, i, j)] = ppm_y(g, qy, i, j, cry[IX(g, i, j)]);
    for (int j = 0; j < n; j++)
        for (int i = -3; i <= n + 2; i++) {
            size_t c = IX(g, i, j), jn = IX(g, i, j + 1);
            qi[c] = (q[c] * area[c] + yfx[c] * fy2[c] - yfx[jn] * fy2[jn]) /
                    (area[c] + yfx[c] - yfx[jn]);
        }
    /* x-direction outer fluxes of q, and the inner advective x update */
    for (int j = -3; j <= n + 2; j++)
        for (int i = 0; i <= n; i++) fx2[IX(g, i, j)] = ppm_x(g, qx, i, j, crx[IX(g, i, j)]);
    for (int j = -3; j <= n + 2; j++)
        for (int i = 0; i < n; i++) {
            size_t c = IX(g, i, j), ie = IX(g, i + 1, j);
            qj[c] = (q[c] * area[c] + xfx[c] * fx2[c] - xfx[ie] * fx2[ie]) /
                    (area[c] + xfx[c] - xfx[ie]);
        }
    /* cross fluxes and the averaged result */
    for (int j = 0; j < n; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j);
            double fx = ppm_x(g, qi, i, j, crx[f]);
            FX[f] = 0.5 * (fx + fx2[f]) * (mx ? mx[f] : xfx[f]);
        }
    for (int j = 0; j <= n; j++)
        for (int i = 0; i < n; i++) {
            size_t f = IX(g, i, j);
            double fy = ppm_y(g, qj, i, j, cry[f]);
            FY[f] = 0.5 * (fy + fy2[f]) * (my ? my[f] : yfx[f]);
        }
    free(fy2); free(fx2); free(qi); free(qj);
}
