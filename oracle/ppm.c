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
 * interval (hord 8).  Three other orders, readings of the un-limited,
 * 2dx-filtered and positive-definite PPM options:
 *  - hord 6, unlimited: the same fourth-order edges and parabola without
 *    either constraint (slopes (q+ - q-)/4, edge deviations unclipped);
 *  - hord 5, 2dx-filtered: the unlimited face, except where the upwind cell
 *    and one of its neighbours are both local extrema (an oscillation over
 *    two cells), where the face takes the upwind cell mean;
 *  - hord 7, positive-definite (tracers): the unlimited parabola of a cell
 *    with a non-negative mean, scaled about that mean by
 *    theta = q / (q - m) when its minimum m over the cell is negative (the
 *    scaling limiter of Zhang and Shu, 2010), so the parabola stays
 *    non-negative and keeps its mean.
 *
 * Tile edges of the cube (option edge_ppm).  Grid lines kink across a cube
 * edge, so the cell edge values next to it are not taken from a stencil that
 * straddles the edge; they come from one-sided extrapolations, as in the
 * panel-edge treatment of Putman & Lin (2007, J. Comput. Phys. 227).  The
 * paper under study is silent on it; the reading used, for a tile edge at
 * interface e (cells e-1 | e) with cell widths dxa along the sweep:
 *  - al(e): the mean of two linear extrapolations to the edge, each through
 *    the centres of the two cells on one side, in physical distance;
 *  - al(e-1) = (3 q(e-1) + 11 q(e-2)) / 14 + (4/7) dm(e-2), from the outer
 *    side only, and al(e+1) = (3 q(e) + 11 q(e+1)) / 14 - (4/7) dm(e+1),
 *    from the inner side only, dm the order's slope (the limited one for
 *    hord 8, the centred one otherwise: then these are the three-cell weights
 *    5/14, 11/14, -2/14);
 *  - hord 5, 6, 7 take these as the cell edge values and go on as usual;
 *  - hord 8, in the two cells beside the edge and in the second cell inside
 *    the tile, leaves the edge deviations unclipped and applies the
 *    monotonicity constraint of Colella & Woodward (1984) instead: flatten
 *    the parabola when the mean is not between its edge values, else move
 *    the edge opposite an interior extremum so the extremum sits on the
 *    cell boundary.
 * Only faces 0, 1, 2 and n-2, n-1, n have an edge cell upwind.  Linear exactness
 * fixes the one-sided weights up to one free parameter; the published value
 * taken for it has no independent check (parity unpinned for that weight).
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

/* cell k of the window is a strict local extremum of its two neighbours */
static int extremum(const double q[6], int k) { return (q[k] - q[k - 1]) * (q[k + 1] - q[k]) < 0.0; }

/* Face value between cells m-1 and m for Courant number c; q[0..5] holds the
 * cells m-3 .. m+2 along the sweep; ord is the PPM order (5, 6, 7 or 8). */
double o_ppm_face_order(const double q[6], double c, int ord)
{
    int s = c > 0.0 ? 2 : 3;   /* the upwind cell (m-1 or m) */
    if (ord == 5 && extremum(q, s) && (extremum(q, s - 1) || extremum(q, s + 1))) return q[s];
    double dm[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 1; k <= 4; k++)
        dm[k] = ord == 8 ? limited_slope(q[k - 1], q[k], q[k + 1]) : (q[k + 1] - q[k - 1]) / 4.0;
    /* left-edge value of cell k (k = 2, 3, 4 are m-1, m, m+1) */
    double al[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 2; k <= 4; k++) al[k] = 0.5 * (q[k - 1] + q[k]) + (dm[k - 1] - dm[k]) / 3.0;
    double bl, br;
    if (ord == 8) {
        bl = -sgn(dm[s]) * min2(2.0 * fabs(dm[s]), fabs(al[s] - q[s]));
        br = sgn(dm[s]) * min2(2.0 * fabs(dm[s]), fabs(al[s + 1] - q[s]));
    } else {
        bl = al[s] - q[s];
        br = al[s + 1] - q[s];
    }
    if (ord == 7 && q[s] >= 0.0) {
        /* minimum of the parabola over the cell: an edge, or the vertex when
         * it is a minimum (a6 < 0) inside the cell (|aR - aL| < -a6) */
        double aL = q[s] + bl, aR = q[s] + br, a6 = -3.0 * (bl + br), da = aR - aL;
        double mn = min2(aL, aR);
        if (a6 < 0.0 && fabs(da) < -a6) mn = min2(mn, q[s] + da * da / (4.0 * a6) + a6 / 12.0);
        if (mn < 0.0) {
            double th = q[s] / (q[s] - mn);
            bl *= th;
            br *= th;
        }
    }
    if (c > 0.0) return q[s] + (1.0 - c) * (br - c * (bl + br));
    return q[s] + (1.0 + c) * (bl + c * (bl + br));
}

double o_ppm_face(const double q[6], double c) { return o_ppm_face_order(q, c, 8); }

/* The face value between window cells 2 and 3 when interface pe of the
 * window (between cells pe-1 and pe, 1 <= pe <= 5) is a tile edge; w[0..5]
 * are the cell widths along the sweep and west is 1 when the tile lies at
 * window cells >= pe, 0 when it lies below pe. */
double o_ppm_face_edge(const double q[6], const double w[6], double c, int ord, int pe, int west)
{
    int s = c > 0.0 ? 2 : 3;
    if (ord == 5 && extremum(q, s) && (extremum(q, s - 1) || extremum(q, s + 1))) return q[s];
    double dm[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 1; k <= 4; k++)
        dm[k] = ord == 8 ? limited_slope(q[k - 1], q[k], q[k + 1]) : (q[k + 1] - q[k - 1]) / 4.0;
    double al[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 2; k <= 4; k++) {
        if (k == pe) {
            /* line through the centres of cells k-2, k-1 (distances w/2 and
             * w(k-1) + w(k-2)/2 below the edge), evaluated at the edge; the
             * same from above through cells k, k+1 */
            double below = ((2.0 * w[k - 1] + w[k - 2]) * q[k - 1] - w[k - 1] * q[k - 2]) / (w[k - 2] + w[k - 1]);
            double above = ((2.0 * w[k] + w[k + 1]) * q[k] - w[k] * q[k + 1]) / (w[k] + w[k + 1]);
            al[k] = 0.5 * (below + above);
        } else if (k == pe - 1) {
            al[k] = (3.0 * q[k] + 11.0 * q[k - 1]) / 14.0 + 4.0 / 7.0 * dm[k - 1];
        } else if (k == pe + 1) {
            al[k] = (3.0 * q[k - 1] + 11.0 * q[k]) / 14.0 - 4.0 / 7.0 * dm[k];
        } else {
            al[k] = 0.5 * (q[k - 1] + q[k]) + (dm[k - 1] - dm[k]) / 3.0;
        }
    }
    int edge_cell = s == pe - 1 || s == pe || s == (west ? pe + 1 : pe - 2);
    double bl, br;
    if (ord == 8 && !edge_cell) {
        bl = -sgn(dm[s]) * min2(2.0 * fabs(dm[s]), fabs(al[s] - q[s]));
        br = sgn(dm[s]) * min2(2.0 * fabs(dm[s]), fabs(al[s + 1] - q[s]));
    } else {
        bl = al[s] - q[s];
        br = al[s + 1] - q[s];
        if (ord == 8) {
            if (bl * br >= 0.0) {
                bl = br = 0.0;   /* the mean is an extremum: flat */
            } else {
                double da = br - bl, a6 = -3.0 * (bl + br);
                if (a6 * da > da * da) bl = -2.0 * br;
                else if (a6 * da < -da * da) br = -2.0 * bl;
            }
        }
    }
    if (ord == 7 && q[s] >= 0.0) {
        double aL = q[s] + bl, aR = q[s] + br, a6 = -3.0 * (bl + br), da = aR - aL;
        double mn = min2(aL, aR);
        if (a6 < 0.0 && fabs(da) < -a6) mn = min2(mn, q[s] + da * da / (4.0 * a6) + a6 / 12.0);
        if (mn < 0.0) {
            double th = q[s] / (q[s] - mn);
            bl *= th;
            br *= th;
        }
    }
    if (c > 0.0) return q[s] + (1.0 - c) * (br - c * (bl + br));
    return q[s] + (1.0 + c) * (bl + c * (bl + br));
}

/* Face m of a sweep of n cells has an edge cell upwind: the window position
 * of the edge and the side the tile lies on.  Only sweeps whose cross index
 * x lies inside the tile take the one-sided values: the sweeps through the
 * corner halo (which feed only the cross-direction updates of halo cells)
 * keep the centred stencil, there being no cell widths in the corner halo. */
static int edge_faces(const OGrid *g, int m, int *pe, int *west)
{
    if (!g->edge_ppm || g->kind != 1) return 0;
    if (m >= 0 && m <= 2) { *pe = 3 - m; *west = 1; return 1; }
    if (m >= g->n - 2 && m <= g->n) { *pe = g->n - m + 3; *west = 0; return 1; }
    return 0;
}
static int edge_window(const OGrid *g, int m, int x, int *pe, int *west)
{
    if (x < 0 || x >= g->n) return 0;
    return edge_faces(g, m, pe, west);
}

/* The kinetic-energy upwinding of d_sw sweeps the D-grid winds along their
 * own rows (u along x, v along y), the cells being the winds' faces with
 * widths dx (dy); its rows 0..n all lie on the tile, so the one-sided edge
 * values apply at faces 0-2 and n-2..n of every row. */
double o_ppm_face_wind(const OGrid *g, const double q[6], const double w[6], double c, int ord, int m)
{
    int pe, west;
    if (edge_faces(g, m, &pe, &west)) return o_ppm_face_edge(q, w, c, ord, pe, west);
    return o_ppm_face_order(q, c, ord);
}

static double ppm_x(const OGrid *g, int t, const double *q, int i, int j, double c, int ord)
{
    double a[6], w[6];
    int pe, west;
    for (int s = 0; s < 6; s++) a[s] = q[IX(g, i - 3 + s, j)];
    if (edge_window(g, i, j, &pe, &west)) {
        const double *dxa = g->dxa + (size_t)t * o_plane(g);
        for (int s = 0; s < 6; s++) w[s] = dxa[IX(g, i - 3 + s, j)];
        return o_ppm_face_edge(a, w, c, ord, pe, west);
    }
    return o_ppm_face_order(a, c, ord);
}
static double ppm_y(const OGrid *g, int t, const double *q, int i, int j, double c, int ord)
{
    double a[6], w[6];
    int pe, west;
    for (int s = 0; s < 6; s++) a[s] = q[IX(g, i, j - 3 + s)];
    if (edge_window(g, j, i, &pe, &west)) {
        const double *dya = g->dya + (size_t)t * o_plane(g);
        for (int s = 0; s < 6; s++) w[s] = dya[IX(g, i, j - 3 + s)];
        return o_ppm_face_edge(a, w, c, ord, pe, west);
    }
    return o_ppm_face_order(a, c, ord);
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
    o_fv_tp_2d_ord(g, g->hord, t, q, qx, qy, crx, cry, xfx, yfx, mx, my, FX, FY);
}

void o_fv_tp_2d_ord(const OGrid *g, int ord, int t, const double *q, const double *qx, const double *qy,
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
        for (int i = -3; i <= n + 2; i++) fy2[IX(g, i, j)] = ppm_y(g, t, qy, i, j, cry[IX(g, i, j)], ord);
    for (int j = 0; j < n; j++)
        for (int i = -3; i <= n + 2; i++) {
            size_t c = IX(g, i, j), jn = IX(g, i, j + 1);
            qi[c] = (q[c] * area[c] + yfx[c] * fy2[c] - yfx[jn] * fy2[jn]) /
                    (area[c] + yfx[c] - yfx[jn]);
        }
    /* x-direction outer fluxes of q, and the inner advective x update */
    for (int j = -3; j <= n + 2; j++)
        for (int i = 0; i <= n; i++) fx2[IX(g, i, j)] = ppm_x(g, t, qx, i, j, crx[IX(g, i, j)], ord);
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
            double fx = ppm_x(g, t, qi, i, j, crx[f], ord);
            FX[f] = 0.5 * (fx + fx2[f]) * (mx ? mx[f] : xfx[f]);
        }
    for (int j = 0; j <= n; j++)
        for (int i = 0; i < n; i++) {
            size_t f = IX(g, i, j);
            double fy = ppm_y(g, t, qj, i, j, cry[f], ord);
            FY[f] = 0.5 * (fy + fy2[f]) * (my ? my[f] : yfx[f]);
        }
    free(fy2); free(fx2); free(qi); free(qj);
}
