/*
 * ORACLE (test infrastructure only): one acoustic substep of the
 * nonhydrostatic FV3 dynamics on Lagrangian surfaces, the substep loop, the
 * tracer transport of the remapping step, and the global mass sums.
 *
 * Sec. II places these loops: the acoustic substep is the innermost loop,
 * with nonblocking halo exchanges of one or more fields at several points in
 * it; tracer advection with the accumulated fluxes belongs to the middle
 * (remapping) loop.  The paper names the modules (c_sw, riem_solver_c,
 * d_sw with fv_tp_2d, riem_solver3) but prints none of their equations
 * except the tile-edge flux rule of Sec. V-B and the corner fill of
 * Sec. VII-C.  Every stage below is therefore a reading of the published
 * C-D grid finite-volume method, stated in the comments, in this order:
 *
 *   H-A   halo of D-grid (u,v) and of delp, pt, w, delz
 *   c_sw  half-step (dt/2) C-grid winds, delp, pt, w
 *   dz_c + riem_solver_c   half-step heights and nonhydrostatic pressure
 *   p_grad_c               C-grid pressure gradient
 *   H-B   halo of C-grid (uc,vc)
 *   d_sw  Courant numbers, fv_tp_2d of delp, pt, w, kinetic energy,
 *         vorticity transport, D-grid momentum update, flux accumulators
 *   dz_d + riem_solver3    heights, vertical velocity and pressure
 *   H-C   halo of pfull, phi, delp
 *   nh_p_grad              D-grid pressure gradient
 */
#include "orc.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PL(f, t, k, K) ((f) + ((size_t)(t) * (K) + (k)) * P)

static double *dalloc(size_t n) { return (double *)calloc(n, sizeof(double)); }
static void fill_nan(double *a, size_t n) { for (size_t s = 0; s < n; s++) a[s] = NAN; }
/* On the cube the corner blocks hold no data; on the periodic grid they do. */
static int skip_corner(const OGrid *g, int st, int i, int j)
{
    return g->kind == 1 && og_region(g, st, i, j) == 2;
}

/* ------------------------------------------- interpolations along a sweep */
/*
 * Along a sweep with interfaces m (interface m between cells m - 1 and m,
 * cell m centred at m + 1/2), x0[(k - m0) s] is the value at index k:
 *  OI_CELL_PT   point value at the centre of cell m from the point values
 *               at the interfaces m - 1 .. m + 2: the cubic's (-1,9,9,-1)/16;
 *  OI_FACE_PT   point value at interface m from the point values at the
 *               centres of cells m - 2 .. m + 1: (-1,9,9,-1)/16;
 *  OI_FACE_MEAN value at interface m from the means of cells m - 2 .. m + 1:
 *               (-1,7,7,-1)/12, the interface value of the cubic whose cell
 *               means they are.
 * With `edge` (the option edge_interp, on sweeps through a cube tile whose
 * tile edges are the interfaces 0 and n), a stencil that would reach across
 * an edge uses only the points on its own side: the interpolant of the
 * three nearest points there (quadratic; for OI_FACE_PT and OI_CELL_PT the
 * weights 3/8, 3/4, -1/8 from the point next to the edge outwards, for
 * OI_FACE_MEAN the cell-mean weights 1/3, 5/6, -1/6), and an interface on
 * the edge itself takes the mean of the two linear extrapolations through
 * the two nearest points (centres, or cell means) of each side,
 * 3/4 (a_{-1} + a_0) - 1/4 (a_{-2} + a_1).  The weights assume evenly spaced
 * points, as the centred ones do.
 */
double o_interp(int kind, const double *x0, ptrdiff_t s, int m0, int m, int n, int edge)
{
#define X(k) x0[(ptrdiff_t)((k) - m0) * s]
    if (kind == OI_CELL_PT) {
        if (edge && (m == 0 || m == n)) return 0.375 * X(m) + 0.75 * X(m + 1) - 0.125 * X(m + 2);
        if (edge && (m == -1 || m == n - 1)) return 0.375 * X(m + 1) + 0.75 * X(m) - 0.125 * X(m - 1);
        return (-X(m - 1) + 9.0 * X(m) + 9.0 * X(m + 1) - X(m + 2)) / 16.0;
    }
    if (edge && (m == 0 || m == n)) return 0.75 * (X(m - 1) + X(m)) - 0.25 * (X(m - 2) + X(m + 1));
    if (kind == OI_FACE_PT) {
        if (edge && (m == 1 || m == n + 1)) return 0.375 * X(m - 1) + 0.75 * X(m) - 0.125 * X(m + 1);
        if (edge && (m == -1 || m == n - 1)) return 0.375 * X(m) + 0.75 * X(m - 1) - 0.125 * X(m - 2);
        return (-X(m - 2) + 9.0 * X(m - 1) + 9.0 * X(m) - X(m + 1)) / 16.0;
    }
    if (edge && (m == 1 || m == n + 1)) return (2.0 * X(m - 1) + 5.0 * X(m) - X(m + 1)) / 6.0;
    if (edge && (m == -1 || m == n - 1)) return (2.0 * X(m) + 5.0 * X(m - 1) - X(m - 2)) / 6.0;
    {
        static const double c4[4] = {-1.0 / 12.0, 7.0 / 12.0, 7.0 / 12.0, -1.0 / 12.0};
        double r = 0.0;
        for (int a = 0; a < 4; a++) r += c4[a] * X(m - 2 + a);
        return r;
    }
#undef X
}

/* Absolute vorticity at corner (i, j) of tile t from the C-grid winds
 * (planes of the tile): f plus the circulation around the dual cell (the
 * four C-grid faces meeting at the corner, each wind times its
 * centre-to-centre length) over the dual-cell area.  At a cube vertex only
 * three cells meet: the two halo faces next to the missing corner cell both
 * cross the single face between the two neighbour cells, so each
 * contributes half. */
double o_corner_vort(const OGrid *g, int t, const double *ucp, const double *vcp, int i, int j)
{
    size_t o = (size_t)t * o_plane(g);
    const double *dxc = g->dxc + o, *dyc = g->dyc + o, *area_c = g->area_c + o, *fB = g->fB + o;
    double ws = 1.0, wn = 1.0, ww = 1.0, we = 1.0;
    if (og_is_vertex(g, i, j)) {
        if (j == 0) ws = 0.5; else wn = 0.5;
        if (i == 0) ww = 0.5; else we = 0.5;
    }
    double circ = ws * ucp[IX(g, i, j - 1)] * dxc[IX(g, i, j - 1)] -
                  wn * ucp[IX(g, i, j)] * dxc[IX(g, i, j)] -
                  ww * vcp[IX(g, i - 1, j)] * dyc[IX(g, i - 1, j)] +
                  we * vcp[IX(g, i, j)] * dyc[IX(g, i, j)];
    return fB[IX(g, i, j)] + circ / area_c[IX(g, i, j)];
}

/* ------------------------------------------------------------------ c_sw */
/*
 * Half-step C-grid update on one level of one tile.  D-grid winds are
 * interpolated to cell centres with (-1,9,9,-1)/16 along the component's own
 * direction and again to the C-grid faces; cell fluxes of delp, pt and w are
 * first-order upwind over dt/2 with the normal wind (u - v cos)/sin; the
 * C-grid winds are advanced by the upwinded absolute-vorticity flux and the
 * kinetic-energy gradient.  Half-step cell quantities are produced on the
 * cells -1..n in both directions (without the four corner cells), so that the
 * C-grid pressure gradient on the interior faces needs no further exchange.
 */
static void c_sw_plane(const OGrid *g, int t, double dt2, const double *u, const double *v,
                       const double *delp, const double *pt, const double *w, double *ucp_out,
                       double *vcp_out, double *delpc, double *ptc, double *wc, double *ax,
                       double *ay, double *vort_out)
{
    int n = g->n;
    size_t P = o_plane(g), o = (size_t)t * P;
    const double *cos_u = g->cos_u + o, *sin_u = g->sin_u + o, *cos_v = g->cos_v + o,
                 *sin_v = g->sin_v + o, *dx = g->dx + o, *dy = g->dy + o, *dxc = g->dxc + o,
                 *dyc = g->dyc + o, *area = g->area + o, *area_c = g->area_c + o,
                 *fB = g->fB + o, *cos_a = g->cos_a + o, *sin_a = g->sin_a + o;
    double *uX = dalloc(P), *vX = dalloc(P), *uY = dalloc(P), *vY = dalloc(P);
    double *ua = dalloc(P), *va = dalloc(P), *uaX = dalloc(P), *vaX = dalloc(P),
           *uaY = dalloc(P), *vaY = dalloc(P);
    double *ucp = dalloc(P), *vcp = dalloc(P), *ke = dalloc(P), *vort = dalloc(P);
    double *dX = dalloc(P), *dY = dalloc(P), *tX = dalloc(P), *tY = dalloc(P), *wX = dalloc(P),
           *wY = dalloc(P);
    double *Fm = dalloc(P), *Fp = dalloc(P), *Fw = dalloc(P), *Gm = dalloc(P), *Gp = dalloc(P),
           *Gw = dalloc(P);
    fill_nan(ua, P); fill_nan(va, P); fill_nan(ucp, P); fill_nan(vcp, P);
    fill_nan(ke, P); fill_nan(vort, P);

    og_view_pair(g, u, ST_Y, v, ST_X, MODE_X, PAIR_SIGNED, uX, vX);
    og_view_pair(g, u, ST_Y, v, ST_X, MODE_Y, PAIR_SIGNED, uY, vY);
    /* one-sided stencils at tile edges only on sweeps whose cross index lies
     * inside the tile (option edge_interp, cube) */
    const int ei = g->edge_interp && g->kind == 1;
    const ptrdiff_t N = g->N;
    /* D -> A: u along y, v along x */
    for (int j = -2; j <= n + 1; j++)
        for (int i = -3; i <= n + 2; i++) {
            if (skip_corner(g, ST_C, i, j)) continue;
            ua[IX(g, i, j)] = o_interp(OI_CELL_PT, uY + IX(g, i, 0), N, 0, j, n, ei && i >= 0 && i < n);
        }
    for (int j = -3; j <= n + 2; j++)
        for (int i = -2; i <= n + 1; i++) {
            if (skip_corner(g, ST_C, i, j)) continue;
            va[IX(g, i, j)] = o_interp(OI_CELL_PT, vX + IX(g, 0, j), 1, 0, i, n, ei && j >= 0 && j < n);
        }
    og_view_pair(g, ua, ST_C, va, ST_C, MODE_X, PAIR_SIGNED, uaX, vaX);
    og_view_pair(g, ua, ST_C, va, ST_C, MODE_Y, PAIR_SIGNED, uaY, vaY);

    /* A -> C on the faces the half-step cells need; normal-wind area fluxes */
    for (int j = -1; j <= n; j++)
        for (int i = -1; i <= n + 1; i++) {
            int inrow = (j >= 0 && j < n);
            if (!inrow && (i < 0 || i > n)) continue;
            size_t f = IX(g, i, j);
            ucp[f] = o_interp(OI_FACE_PT, uaX + IX(g, 0, j), 1, 0, i, n, ei && inrow);
            ax[f] = dt2 * (ucp[f] - v[f] * cos_u[f]) / sin_u[f] * dy[f];
        }
    for (int j = -1; j <= n + 1; j++)
        for (int i = -1; i <= n; i++) {
            int incol = (i >= 0 && i < n);
            if (!incol && (j < 0 || j > n)) continue;
            size_t f = IX(g, i, j);
            vcp[f] = o_interp(OI_FACE_PT, vaY + IX(g, i, 0), N, 0, j, n, ei && incol);
            ay[f] = dt2 * (vcp[f] - u[f] * cos_v[f]) / sin_v[f] * dx[f];
        }

    /* first-order upwind fluxes of delp, pt*delp, w*delp */
    og_view_scalar(g, delp, ST_C, MODE_X, 0, dX);
    og_view_scalar(g, delp, ST_C, MODE_Y, 0, dY);
    og_view_scalar(g, pt, ST_C, MODE_X, 0, tX);
    og_view_scalar(g, pt, ST_C, MODE_Y, 0, tY);
    og_view_scalar(g, w, ST_C, MODE_X, 0, wX);
    og_view_scalar(g, w, ST_C, MODE_Y, 0, wY);
    for (int j = -1; j <= n; j++)
        for (int i = -1; i <= n + 1; i++) {
            int inrow = (j >= 0 && j < n);
            if (!inrow && (i < 0 || i > n)) continue;
            size_t f = IX(g, i, j), up = ax[f] > 0.0 ? IX(g, i - 1, j) : f;
            Fm[f] = ax[f] * dX[up];
            Fp[f] = Fm[f] * tX[up];
            Fw[f] = Fm[f] * wX[up];
        }
    for (int j = -1; j <= n + 1; j++)
        for (int i = -1; i <= n; i++) {
            int incol = (i >= 0 && i < n);
            if (!incol && (j < 0 || j > n)) continue;
            size_t f = IX(g, i, j), up = ay[f] > 0.0 ? IX(g, i, j - 1) : f;
            Gm[f] = ay[f] * dY[up];
            Gp[f] = Gm[f] * tY[up];
            Gw[f] = Gm[f] * wY[up];
        }
    for (int j = -1; j <= n; j++)
        for (int i = -1; i <= n; i++) {
            int cross = (i >= 0 && i < n) || (j >= 0 && j < n);
            if (!cross) continue;
            size_t c = IX(g, i, j), e = IX(g, i + 1, j), nn = IX(g, i, j + 1);
            delpc[c] = delp[c] + (Fm[c] - Fm[e] + Gm[c] - Gm[nn]) / area[c];
            ptc[c] = (pt[c] * delp[c] + (Fp[c] - Fp[e] + Gp[c] - Gp[nn]) / area[c]) / delpc[c];
            wc[c] = (w[c] * delp[c] + (Fw[c] - Fw[e] + Gw[c] - Gw[nn]) / area[c]) / delpc[c];
            /* kinetic energy at the centre, upwinded with the contravariant wind */
            double s2 = sin_a[c] * sin_a[c];
            double uac = (ua[c] - va[c] * cos_a[c]) / s2;
            double vac = (va[c] - ua[c] * cos_a[c]) / s2;
            ke[c] = 0.5 * dt2 * (uac * (uac > 0.0 ? ucp[c] : ucp[e]) +
                                 vac * (vac > 0.0 ? vcp[c] : vcp[nn]));
        }

    /* absolute vorticity at corners from the C-grid circulation */
    for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            size_t b = IX(g, i, j);
            vort[b] = o_corner_vort(g, t, ucp, vcp, i, j);
            if (vort_out) vort_out[b] = vort[b];
        }

    /* C-grid wind update on the interior faces */
    for (int j = 0; j < n; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j);
            double fy1 = dt2 * (v[f] - ucp[f] * cos_u[f]) / sin_u[f];
            double vt = fy1 > 0.0 ? vort[IX(g, i, j)] : vort[IX(g, i, j + 1)];
            ucp_out[f] = ucp[f] + fy1 * vt + (ke[IX(g, i - 1, j)] - ke[f]) / dxc[f];
        }
    for (int j = 0; j <= n; j++)
        for (int i = 0; i < n; i++) {
            size_t f = IX(g, i, j);
            double fx1 = dt2 * (u[f] - vcp[f] * cos_v[f]) / sin_v[f];
            double vt = fx1 > 0.0 ? vort[IX(g, i, j)] : vort[IX(g, i + 1, j)];
            vcp_out[f] = vcp[f] - fx1 * vt + (ke[IX(g, i, j - 1)] - ke[f]) / dyc[f];
        }
    double *fr[] = {uX, vX, uY, vY, ua, va, uaX, vaX, uaY, vaY, ucp, vcp, ke, vort, dX, dY,
                    tX, tY, wX, wY, Fm, Fp, Fw, Gm, Gp, Gw};
    for (size_t q = 0; q < sizeof(fr) / sizeof(fr[0]); q++) free(fr[q]);
}

/* heights at interfaces from the layer thicknesses: zh[nz] = surface, upward sum */
static void heights(const OGrid *g, int t, const double *delz, const double *zs, double *zh)
{
    int nz = g->nz;
    size_t P = o_plane(g);
    for (int s = 0; s < (int)P; s++) {
        zh[(size_t)nz * P + s] = zs[s];
        for (int k = nz - 1; k >= 0; k--)
            zh[(size_t)k * P + s] = zh[(size_t)(k + 1) * P + s] - delz[((size_t)t * nz + k) * P + s];
    }
}

/* ------------------------------------------- dz_c + riem_solver_c (one tile) */
/*
 * Half-step interface heights: each interface is moved by first-order upwind
 * transport with the area fluxes of the two adjacent layers averaged (the top
 * interface takes the top layer's), in advective form; the surface is fixed.
 * The semi-implicit column solve over dt/2 then gives the half-step interface
 * pressure and geopotential used by the C-grid pressure gradient.
 */
/* virtual potential temperature factor 1 + (Rv/Rd - 1) q of a layer */
static double o_virt(const double *qv, size_t idx)
{
    return qv ? 1.0 + (O_RVGAS / O_RDGAS - 1.0) * qv[idx] : 1.0;
}

static void dzc_riemc_tile(const OGrid *g, int t, double dt2, const double *delz,
                           const double *zs, const double *ax, const double *ay,
                           const double *delpc, const double *ptc, const double *wc,
                           const double *qv, double *pkc, double *gz)
{
    int n = g->n, nz = g->nz;
    size_t P = o_plane(g), o = (size_t)t * P;
    const double *area = g->area + o;
    double *zh = dalloc((size_t)(nz + 1) * P);
    double *zhX = dalloc((size_t)(nz + 1) * P), *zhY = dalloc((size_t)(nz + 1) * P);
    heights(g, t, delz, zs, zh);
    for (int K = 0; K <= nz; K++) {
        og_view_scalar(g, zh + (size_t)K * P, ST_C, MODE_X, 0, zhX + (size_t)K * P);
        og_view_scalar(g, zh + (size_t)K * P, ST_C, MODE_Y, 0, zhY + (size_t)K * P);
    }
    double *col_d = dalloc(nz), *col_t = dalloc(nz), *col_w = dalloc(nz), *col_z = dalloc(nz);
    double *wo = dalloc(nz), *dzo = dalloc(nz), *pf = dalloc(nz + 1), *ph = dalloc(nz + 1);
    double *zc = dalloc(nz + 1);
#define AXL(K, f) ((K) == 0 ? PL(ax, t, 0, nz)[f] : 0.5 * (PL(ax, t, (K) - 1, nz)[f] + PL(ax, t, (K), nz)[f]))
#define AYL(K, f) ((K) == 0 ? PL(ay, t, 0, nz)[f] : 0.5 * (PL(ay, t, (K) - 1, nz)[f] + PL(ay, t, (K), nz)[f]))
    for (int j = -1; j <= n; j++)
        for (int i = -1; i <= n; i++) {
            int cross = (i >= 0 && i < n) || (j >= 0 && j < n);
            if (!cross) continue;
            size_t c = IX(g, i, j), w_ = IX(g, i - 1, j), e = IX(g, i + 1, j), s = IX(g, i, j - 1),
                   nn = IX(g, i, j + 1);
            for (int K = 0; K < nz; K++) {
                const double *zx = zhX + (size_t)K * P, *zy = zhY + (size_t)K * P;
                double a0 = AXL(K, c), a1 = AXL(K, e), b0 = AYL(K, c), b1 = AYL(K, nn);
                double z0 = a0 > 0.0 ? zx[w_] : zx[c];
                double z1 = a1 > 0.0 ? zx[c] : zx[e];
                double y0 = b0 > 0.0 ? zy[s] : zy[c];
                double y1 = b1 > 0.0 ? zy[c] : zy[nn];
                zc[K] = (zh[(size_t)K * P + c] * area[c] + a0 * z0 - a1 * z1 + b0 * y0 - b1 * y1) /
                        (area[c] + a0 - a1 + b0 - b1);
            }
            zc[nz] = zs[c];
            for (int k = 0; k < nz; k++) {
                col_z[k] = zc[k + 1] - zc[k];
                col_d[k] = PL(delpc, t, k, nz)[c];
                col_t[k] = PL(ptc, t, k, nz)[c] * o_virt(qv, (size_t)(t * nz + k) * P + c);
                col_w[k] = PL(wc, t, k, nz)[c];
            }
            o_sim1b(nz, dt2, g->beta, g->pp_order, g->ptop, zs[c], col_d, col_t, col_z, col_w, wo, dzo, pf, ph, 0, 0);
            for (int K = 0; K <= nz; K++) {
                PL(pkc, t, K, nz + 1)[c] = pf[K];
                PL(gz, t, K, nz + 1)[c] = ph[K];
            }
        }
#undef AXL
#undef AYL
    free(zh); free(zhX); free(zhY); free(col_d); free(col_t); free(col_w); free(col_z);
    free(wo); free(dzo); free(pf); free(ph); free(zc);
}

/* ----------------------------------------------------------- p_grad_c */
static void pgradc_plane(const OGrid *g, int t, int k, double dt2, const double *delpc,
                         const double *pkc, const double *gz, double *uc, double *vc)
{
    int n = g->n, nz = g->nz;
    size_t P = o_plane(g), o = (size_t)t * P;
    const double *dp = PL(delpc, t, k, nz);
    const double *p0 = PL(pkc, t, k, nz + 1), *p1 = PL(pkc, t, k + 1, nz + 1);
    const double *z0 = PL(gz, t, k, nz + 1), *z1 = PL(gz, t, k + 1, nz + 1);
    double *U = PL(uc, t, k, nz), *V = PL(vc, t, k, nz);
    for (int j = 0; j < n; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j), W = IX(g, i - 1, j), E = f;
            U[f] += o_pgf(dt2, g->dxc[o + f], dp[W], dp[E], z0[W], z1[W], z0[E], z1[E], p0[W],
                          p1[W], p0[E], p1[E]);
        }
    for (int j = 0; j <= n; j++)
        for (int i = 0; i < n; i++) {
            size_t f = IX(g, i, j), W = IX(g, i, j - 1), E = f;
            V[f] += o_pgf(dt2, g->dyc[o + f], dp[W], dp[E], z0[W], z1[W], z0[E], z1[E], p0[W],
                          p1[W], p0[E], p1[E]);
        }
}

/* --------------------------------------------------------------- d_sw */
/*
 * Full-step D-grid update on one level of one tile.  Courant numbers and area
 * fluxes come from the contravariant half-step C-grid winds (the tangential
 * partner is the four-point mean of the other C-grid component); delp is
 * transported by fv_tp_2d, pt and w by fv_tp_2d weighted with its mass
 * fluxes; the kinetic energy at corners upwinds D-grid u along x and v along
 * y by PPM with the corner displacements; absolute vorticity at cells is
 * transported by fv_tp_2d and its fluxes, with the kinetic-energy
 * differences, update the D-grid winds.
 */
/*
 * Smagorinsky magnitude at the corners of one level of tile t:
 * dt sqrt(DT^2 + DS^2) (the expression the paper quotes for its Smagorinsky
 * kernel, Sec. VII-C), with the deformation of the D-grid winds in finite
 * volume form: tension DT = du/dx - dv/dy at the corner from the normal
 * components through the four edges of its dual cell (the divergence's terms
 * with the v part negated; at a cube vertex the two edges next to the missing
 * cell count half), shear DS = dv/dx + du/dy at the cells from the tangential
 * components around each cell (the vorticity's terms with the u part
 * negated), averaged to the corner over its four cells (three at a cube
 * vertex).  u, v need their halos.
 */
void o_smag_corner(const OGrid *g, int t, const double *u, const double *v, double dt, double *out)
{
    const int n = g->n;
    const size_t o = (size_t)t * o_plane(g);
    const double *dx = g->dx + o, *dy = g->dy + o, *dxc = g->dxc + o, *dyc = g->dyc + o;
    const double *area = g->area + o, *area_c = g->area_c + o;
    double *shear = (double *)calloc(o_plane(g), sizeof(double));
    for (int j = -1; j <= n; j++)
        for (int i = -1; i <= n; i++) {
            if (skip_corner(g, ST_C, i, j)) continue;
            size_t c = IX(g, i, j);
            shear[c] = (v[IX(g, i + 1, j)] * dy[IX(g, i + 1, j)] - v[c] * dy[c] +
                        u[IX(g, i, j + 1)] * dx[IX(g, i, j + 1)] - u[c] * dx[c]) / area[c];
        }
    for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            size_t b = IX(g, i, j);
            double ws = 1.0, wn = 1.0, ww = 1.0, we = 1.0;
            if (og_is_vertex(g, i, j)) {
                if (j == 0) ws = 0.5; else wn = 0.5;
                if (i == 0) ww = 0.5; else we = 0.5;
            }
            double tension = (we * u[b] * dyc[b] - ww * u[IX(g, i - 1, j)] * dyc[IX(g, i - 1, j)] -
                              wn * v[b] * dxc[b] + ws * v[IX(g, i, j - 1)] * dxc[IX(g, i, j - 1)]) / area_c[b];
            double s = 0.0;
            int cnt = 0;
            for (int dj = -1; dj <= 0; dj++)
                for (int di = -1; di <= 0; di++) {
                    if (skip_corner(g, ST_C, i + di, j + dj)) continue;
                    s += shear[IX(g, i + di, j + dj)];
                    cnt++;
                }
            double sh = s / cnt;
            out[b] = dt * sqrt(tension * tension + sh * sh);
        }
    free(shear);
}

/* Edge-flux fix-up on the cube.  A face on a tile edge is stored by both
 * tiles and each computes its own flux through it; both fluxes are replaced
 * by their mean (the partner's counted along our direction), and the cell
 * next to the face takes the difference, so that what leaves one tile enters
 * the other.  edge_faces lists, for cell (i, j) of a tile, its faces on the
 * tile edge: stagger, face indices and the sign with which a flux along +x or
 * +y enters the cell. */
static int edge_faces(const OGrid *g, int i, int j, int st[2], int fi[2], int fj[2], int sg[2])
{
    int n = g->n, m = 0;
    if (i == 0) { st[m] = ST_X; fi[m] = 0; fj[m] = j; sg[m] = 1; m++; }
    if (i == n - 1) { st[m] = ST_X; fi[m] = n; fj[m] = j; sg[m] = -1; m++; }
    if (j == 0) { st[m] = ST_Y; fi[m] = i; fj[m] = 0; sg[m] = 1; m++; }
    if (j == n - 1) { st[m] = ST_Y; fi[m] = i; fj[m] = n; sg[m] = -1; m++; }
    return m;
}

/* the mean flux through a shared face minus our own, for one quantity */
static double edge_delta(const OGrid *g, int nlev, const double *FX, const double *FY, int t, int k, int st,
                         int i, int j)
{
    size_t P = o_plane(g);
    int tp, stp, ip, jp;
    int sg = og_edge_partner(g, t, st, i, j, &tp, &stp, &ip, &jp);
    const double *own = st == ST_X ? FX : FY, *par = stp == ST_X ? FX : FY;
    double fo = own[((size_t)t * nlev + k) * P + IX(g, i, j)];
    double fp = sg * par[((size_t)tp * nlev + k) * P + IX(g, ip, jp)];
    return 0.5 * (fo + fp) - fo;
}

void o_edge_fix_dsw(const OGrid *g, const double *FXm, const double *FYm, const double *FXp,
                    const double *FYp, const double *FXw, const double *FYw, double *delp, double *pt,
                    double *w, double *mfx, double *mfy)
{
    int n = g->n, nz = g->nz;
    size_t P = o_plane(g);
    if (g->kind != 1) return;
    /* all deltas from the unmodified fluxes first, then the updates */
    size_t F3 = (size_t)g->T * nz * P;
    double *dM = dalloc(F3), *dP = dalloc(F3), *dW = dalloc(F3);
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    int st[2], fi[2], fj[2], sg[2];
                    int m = edge_faces(g, i, j, st, fi, fj, sg);
                    size_t c = PL(dM, t, k, nz) - dM + IX(g, i, j);
                    for (int q = 0; q < m; q++) {
                        double em = edge_delta(g, nz, FXm, FYm, t, k, st[q], fi[q], fj[q]);
                        dM[c] += sg[q] * em;
                        dP[c] += sg[q] * edge_delta(g, nz, FXp, FYp, t, k, st[q], fi[q], fj[q]);
                        dW[c] += sg[q] * edge_delta(g, nz, FXw, FYw, t, k, st[q], fi[q], fj[q]);
                        double *acc = st[q] == ST_X ? mfx : mfy;
                        acc[PL(acc, t, k, nz) - acc + IX(g, fi[q], fj[q])] += em;
                    }
                }
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    if (i > 0 && i < n - 1 && j > 0 && j < n - 1) continue;
                    size_t c = PL(dM, t, k, nz) - dM + IX(g, i, j);
                    double a = g->area[(size_t)t * P + IX(g, i, j)];
                    double d0 = delp[c], d1 = d0 + dM[c] / a;
                    pt[c] = (pt[c] * d0 * a + dP[c]) / (d1 * a);
                    w[c] = (w[c] * d0 * a + dW[c]) / (d1 * a);
                    delp[c] = d1;
                }
    free(dM); free(dP); free(dW);
}

void o_edge_fix_tracer(const OGrid *g, const double *FX, const double *FY, const double *dp2, double *q)
{
    int n = g->n, nz = g->nz;
    size_t P = o_plane(g);
    if (g->kind != 1) return;
    size_t F3 = (size_t)g->T * nz * P;
    double *dQ = dalloc(F3);
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    int st[2], fi[2], fj[2], sg[2];
                    int m = edge_faces(g, i, j, st, fi, fj, sg);
                    size_t c = PL(dQ, t, k, nz) - dQ + IX(g, i, j);
                    for (int r = 0; r < m; r++) dQ[c] += sg[r] * edge_delta(g, nz, FX, FY, t, k, st[r], fi[r], fj[r]);
                }
    for (size_t c = 0; c < F3; c++)
        if (dQ[c] != 0.0) q[c] += dQ[c] / (dp2[c] * g->area[(c / ((size_t)nz * P)) * P + c % P]);
    free(dQ);
}

/* Divergence at the corners 0..n of a D-grid pair (U on y-faces, V on
 * x-faces) over each corner's dual cell: normal components through its four
 * edges times their lengths over the dual area; at a cube vertex the two
 * edges next to the missing cell count half. */
void o_corner_div(const OGrid *g, int t, const double *U, const double *V, double *out)
{
    int n = g->n;
    size_t o = (size_t)t * o_plane(g);
    const double *dxc = g->dxc + o, *dyc = g->dyc + o, *area_c = g->area_c + o;
    for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            size_t b = IX(g, i, j);
            double ws = 1.0, wn = 1.0, ww = 1.0, we = 1.0;
            if (og_is_vertex(g, i, j)) {
                if (j == 0) ws = 0.5; else wn = 0.5;
                if (i == 0) ww = 0.5; else we = 0.5;
            }
            out[b] = (we * U[b] * dyc[b] - ww * U[IX(g, i - 1, j)] * dyc[IX(g, i - 1, j)] +
                      wn * V[b] * dxc[b] - ws * V[IX(g, i, j - 1)] * dxc[IX(g, i, j - 1)]) / area_c[b];
        }
}

/* Corner Laplacian of a corner field D (its halo filled): the corner
 * divergence of its gradient along the cell edges, (D(i+1,j) - D(i,j)) / dx
 * on y-faces and (D(i,j+1) - D(i,j)) / dy on x-faces. */
void o_corner_lap(const OGrid *g, int t, const double *D, double *out)
{
    int n = g->n;
    size_t P = o_plane(g), o = (size_t)t * P;
    const double *dx = g->dx + o, *dy = g->dy + o;
    double *GU = (double *)calloc(P, sizeof(double)), *GV = (double *)calloc(P, sizeof(double));
    for (int j = 0; j <= n; j++)
        for (int i = -1; i <= n; i++) {
            size_t f = IX(g, i, j);
            GU[f] = (D[IX(g, i + 1, j)] - D[f]) / dx[f];
        }
    for (int j = -1; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j);
            GV[f] = (D[IX(g, i, j + 1)] - D[f]) / dy[f];
        }
    o_corner_div(g, t, GU, GV, out);
    free(GU);
    free(GV);
}

static void d_sw_plane(const OGrid *g, int t, int k, double bdt, double *u, double *v,
                       const double *uc, const double *vc, double *delp, double *pt, double *w,
                       double *mfx, double *mfy, double *cx, double *cy, double *crx,
                       double *cry, double *xfx, double *yfx, const double *hd, double *const *ef, int *cfl,
                       double *om_out)
{
    int n = g->n;
    size_t P = o_plane(g), o = (size_t)t * P;
    const double *cos_u = g->cos_u + o, *sin_u = g->sin_u + o, *cos_v = g->cos_v + o,
                 *sin_v = g->sin_v + o, *dx = g->dx + o, *dy = g->dy + o, *area = g->area + o,
                 *fC = g->fC + o;
    double *dxaX = dalloc(P), *dyaX = dalloc(P), *dxaY = dalloc(P), *dyaY = dalloc(P);
    double *ucX = dalloc(P), *vcX = dalloc(P), *ucY = dalloc(P), *vcY = dalloc(P);
    double *ut = dalloc(P), *vt = dalloc(P);
    double *qx = dalloc(P), *qy = dalloc(P);
    double *FX = dalloc(P), *FY = dalloc(P), *GX = dalloc(P), *GY = dalloc(P);
    double *ke = dalloc(P), *om = dalloc(P), *VX = dalloc(P), *VY = dalloc(P);
    double *dn = dalloc(P), *pn = dalloc(P), *wn = dalloc(P);
    fill_nan(ut, P); fill_nan(vt, P); fill_nan(om, P);

    og_view_pair(g, g->dxa + o, ST_C, g->dya + o, ST_C, MODE_X, PAIR_ABS, dxaX, dyaX);
    og_view_pair(g, g->dxa + o, ST_C, g->dya + o, ST_C, MODE_Y, PAIR_ABS, dxaY, dyaY);
    og_view_pair(g, uc, ST_X, vc, ST_Y, MODE_X, PAIR_SIGNED, ucX, vcX);
    og_view_pair(g, uc, ST_X, vc, ST_Y, MODE_Y, PAIR_SIGNED, ucY, vcY);

    /* (i) Courant numbers and area fluxes */
    for (int j = -3; j <= n + 2; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j);
            double vb = 0.25 * (vcX[IX(g, i - 1, j)] + vcX[f] + vcX[IX(g, i - 1, j + 1)] +
                                vcX[IX(g, i, j + 1)]);
            ut[f] = (uc[f] - vb * cos_u[f]) / (sin_u[f] * sin_u[f]);
            size_t up = ut[f] > 0.0 ? IX(g, i - 1, j) : f;
            crx[f] = bdt * ut[f] / dxaX[up];
            xfx[f] = bdt * ut[f] * sin_u[f] * dy[f];
            if (fabs(crx[f]) > 1.0) *cfl = 1;
        }
    for (int j = 0; j <= n; j++)
        for (int i = -3; i <= n + 2; i++) {
            size_t f = IX(g, i, j);
            double ub = 0.25 * (ucY[IX(g, i, j - 1)] + ucY[IX(g, i + 1, j - 1)] + ucY[f] +
                                ucY[IX(g, i + 1, j)]);
            vt[f] = (vc[f] - ub * cos_v[f]) / (sin_v[f] * sin_v[f]);
            size_t up = vt[f] > 0.0 ? IX(g, i, j - 1) : f;
            cry[f] = bdt * vt[f] / dyaY[up];
            yfx[f] = bdt * vt[f] * sin_v[f] * dx[f];
            if (fabs(cry[f]) > 1.0) *cfl = 1;
        }

    /* (ii) mass: delp */
    og_view_scalar(g, delp, ST_C, MODE_X, 0, qx);
    og_view_scalar(g, delp, ST_C, MODE_Y, 0, qy);
    o_fv_tp_2d(g, t, delp, qx, qy, crx, cry, xfx, yfx, NULL, NULL, FX, FY);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            size_t c = IX(g, i, j);
            dn[c] = delp[c] + (FX[c] - FX[IX(g, i + 1, j)] + FY[c] - FY[IX(g, i, j + 1)]) / area[c];
        }
    /* fluxes kept for the edge-flux fix-up */
    if (ef) {
        memcpy(ef[0], FX, P * sizeof(double));
        memcpy(ef[1], FY, P * sizeof(double));
    }
    /* (iii) pt and w with the mass fluxes */
    og_view_scalar(g, pt, ST_C, MODE_X, 0, qx);
    og_view_scalar(g, pt, ST_C, MODE_Y, 0, qy);
    o_fv_tp_2d(g, t, pt, qx, qy, crx, cry, xfx, yfx, FX, FY, GX, GY);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            size_t c = IX(g, i, j);
            pn[c] = (pt[c] * delp[c] * area[c] + GX[c] - GX[IX(g, i + 1, j)] + GY[c] -
                     GY[IX(g, i, j + 1)]) / (dn[c] * area[c]);
        }
    if (ef) {
        memcpy(ef[2], GX, P * sizeof(double));
        memcpy(ef[3], GY, P * sizeof(double));
    }
    og_view_scalar(g, w, ST_C, MODE_X, 0, qx);
    og_view_scalar(g, w, ST_C, MODE_Y, 0, qy);
    o_fv_tp_2d(g, t, w, qx, qy, crx, cry, xfx, yfx, FX, FY, GX, GY);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            size_t c = IX(g, i, j);
            wn[c] = (w[c] * delp[c] * area[c] + GX[c] - GX[IX(g, i + 1, j)] + GY[c] -
                     GY[IX(g, i, j + 1)]) / (dn[c] * area[c]);
        }
    if (ef) {
        memcpy(ef[4], GX, P * sizeof(double));
        memcpy(ef[5], GY, P * sizeof(double));
    }
    /* (iv) accumulate mass fluxes and Courant numbers on the interior faces */
    for (int j = 0; j < n; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j);
            mfx[f] += FX[f];
            cx[f] += crx[f];
        }
    for (int j = 0; j <= n; j++)
        for (int i = 0; i < n; i++) {
            size_t f = IX(g, i, j);
            mfy[f] += FY[f];
            cy[f] += cry[f];
        }
    /* (v) kinetic energy at corners */
    for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            size_t b = IX(g, i, j);
            double ub = 0.5 * bdt * (ut[IX(g, i, j - 1)] + ut[b]);
            double vb = 0.5 * bdt * (vt[IX(g, i - 1, j)] + vt[b]);
            double a6[6], w6[6];
            double cxu = ub / dx[ub > 0.0 ? IX(g, i - 1, j) : b];
            for (int s = 0; s < 6; s++) {
                a6[s] = u[IX(g, i - 3 + s, j)];
                w6[s] = dx[IX(g, i - 3 + s, j)];
            }
            double ubv = o_ppm_face_wind(g, a6, w6, cxu, g->hord, i);
            double cyv = vb / dy[vb > 0.0 ? IX(g, i, j - 1) : b];
            for (int s = 0; s < 6; s++) {
                a6[s] = v[IX(g, i, j - 3 + s)];
                w6[s] = dy[IX(g, i, j - 3 + s)];
            }
            double vbv = o_ppm_face_wind(g, a6, w6, cyv, g->hord, j);
            ke[b] = 0.5 * (ub * ubv + vb * vbv);
        }
    /* (v') optional del-2 divergence damping: nu times the divergence of the
     * D-grid winds over the dual cell of each corner (normal components
     * through the four dual edges; at a cube vertex the two edges next to the
     * missing cell count half) is subtracted from the kinetic energy, so that
     * the wind update below adds nu times its gradient: a diffusion of the
     * divergence with coefficient nu = d2_bg times the smallest dual-cell area */
    if (g->d2_bg > 0.0 || g->dddmp > 0.0) {
        const double *dxc = g->dxc + o, *dyc = g->dyc + o, *area_c = g->area_c + o;
        double *smag = NULL;
        if (g->dddmp > 0.0) {
            smag = (double *)calloc(o_plane(g), sizeof(double));
            o_smag_corner(g, t, u, v, bdt, smag);
        }
        for (int j = 0; j <= n; j++)
            for (int i = 0; i <= n; i++) {
                size_t b = IX(g, i, j);
                /* coefficient: d2_bg, raised by the Smagorinsky magnitude up to 0.2 */
                double c2 = g->d2_bg;
                if (smag) {
                    double cs = g->dddmp * smag[b];
                    if (cs > 0.2) cs = 0.2;
                    if (cs > c2) c2 = cs;
                }
                double nu = c2 * g->da_min;
                double ws = 1.0, wn = 1.0, ww = 1.0, we = 1.0;
                if (og_is_vertex(g, i, j)) {
                    if (j == 0) ws = 0.5; else wn = 0.5;
                    if (i == 0) ww = 0.5; else we = 0.5;
                }
                double flux = we * u[b] * dyc[b] - ww * u[IX(g, i - 1, j)] * dyc[IX(g, i - 1, j)] +
                              wn * v[b] * dxc[b] - ws * v[IX(g, i, j - 1)] * dxc[IX(g, i, j - 1)];
                ke[b] -= nu * flux / area_c[b];
            }
        free(smag);
    }
    /* (v'') optional higher-order divergence damping: hd holds the corner
     * divergence with nord corner Laplacians applied; (-1)^(nord+1) nu_n hd is
     * added to the kinetic energy, nu_n = (d4_bg da_min)^(nord+1), so that the
     * divergence obeys dD/dt = (-1)^nord nu_n Lap^(nord+1) D (del-4: nord = 1,
     * del-6: nord = 2) */
    if (hd) {
        double nun = pow(g->d4_bg * g->da_min, g->nord + 1);
        double sg = (g->nord % 2) ? 1.0 : -1.0;
        for (int j = 0; j <= n; j++)
            for (int i = 0; i <= n; i++) ke[IX(g, i, j)] += sg * nun * hd[IX(g, i, j)];
    }
    /* (vi) absolute vorticity at cells and its transport */
    for (int j = -3; j <= n + 2; j++)
        for (int i = -3; i <= n + 2; i++) {
            if (skip_corner(g, ST_C, i, j)) continue;
            size_t c = IX(g, i, j);
            om[c] = fC[c] + (u[c] * dx[c] - u[IX(g, i, j + 1)] * dx[IX(g, i, j + 1)] -
                             v[c] * dy[c] + v[IX(g, i + 1, j)] * dy[IX(g, i + 1, j)]) / area[c];
            if (om_out && i >= 0 && i < n && j >= 0 && j < n) om_out[c] = om[c];
        }
    og_view_scalar(g, om, ST_C, MODE_X, 0, qx);
    og_view_scalar(g, om, ST_C, MODE_Y, 0, qy);
    o_fv_tp_2d(g, t, om, qx, qy, crx, cry, xfx, yfx, NULL, NULL, VX, VY);
    /* (vii) optional del-2 vorticity damping: a diffusive flux of the
     * relative vorticity joins the vorticity fluxes, nu_v times its
     * difference across the face over the centre distance times the face
     * length (into the cell on the low side), so that the vorticity of the
     * updated winds diffuses with nu_v = vtdm times the smallest dual area */
    if (g->vtdm > 0.0) {
        double nuv = g->vtdm * g->da_min;
        const double *dxc = g->dxc + o, *dyc = g->dyc + o;
        for (int j = 0; j < n; j++)
            for (int i = 0; i <= n; i++) {
                size_t f = IX(g, i, j), w_ = IX(g, i - 1, j);
                VX[f] += nuv * ((om[w_] - fC[w_]) - (om[f] - fC[f])) * dy[f] / dxc[f];
            }
        for (int j = 0; j <= n; j++)
            for (int i = 0; i < n; i++) {
                size_t f = IX(g, i, j), s_ = IX(g, i, j - 1);
                VY[f] += nuv * ((om[s_] - fC[s_]) - (om[f] - fC[f])) * dx[f] / dyc[f];
            }
    }
    /* (viii) D-grid wind update (pressure gradient follows after riem_solver3) */
    for (int j = 0; j <= n; j++)
        for (int i = 0; i < n; i++) {
            size_t f = IX(g, i, j);
            u[f] = u[f] + (ke[f] - ke[IX(g, i + 1, j)] + VY[f]) / dx[f];
        }
    for (int j = 0; j < n; j++)
        for (int i = 0; i <= n; i++) {
            size_t f = IX(g, i, j);
            v[f] = v[f] + (ke[f] - ke[IX(g, i, j + 1)] - VX[f]) / dy[f];
        }
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            size_t c = IX(g, i, j);
            delp[c] = dn[c]; pt[c] = pn[c]; w[c] = wn[c];
        }
    (void)k;
    double *fr[] = {dxaX, dyaX, dxaY, dyaY, ucX, vcX, ucY, vcY, ut, vt, qx, qy, FX, FY, GX, GY,
                    ke, om, VX, VY, dn, pn, wn};
    for (size_t q = 0; q < sizeof(fr) / sizeof(fr[0]); q++) free(fr[q]);
}

/* --------------------------------------------------- dz_d (one tile) */
/*
 * Interface heights transported by fv_tp_2d with the Courant numbers and area
 * fluxes of the adjacent layers averaged (top interface: top layer), in
 * advective form; the surface stays fixed.  New thicknesses follow.
 */
static void dzd_tile(const OGrid *g, int t, double *delz, const double *zs, const double *crx,
                     const double *cry, const double *xfx, const double *yfx)
{
    int n = g->n, nz = g->nz;
    size_t P = o_plane(g), o = (size_t)t * P;
    const double *area = g->area + o;
    double *zh = dalloc((size_t)(nz + 1) * P), *zn = dalloc((size_t)(nz + 1) * P);
    double *qx = dalloc(P), *qy = dalloc(P), *ZX = dalloc(P), *ZY = dalloc(P);
    double *cxI = dalloc(P), *cyI = dalloc(P), *xI = dalloc(P), *yI = dalloc(P);
    heights(g, t, delz, zs, zh);
    for (int K = 0; K < nz; K++) {
        const double *a0 = PL(crx, t, K == 0 ? 0 : K - 1, nz), *a1 = PL(crx, t, K, nz);
        const double *b0 = PL(cry, t, K == 0 ? 0 : K - 1, nz), *b1 = PL(cry, t, K, nz);
        const double *c0 = PL(xfx, t, K == 0 ? 0 : K - 1, nz), *c1 = PL(xfx, t, K, nz);
        const double *d0 = PL(yfx, t, K == 0 ? 0 : K - 1, nz), *d1 = PL(yfx, t, K, nz);
        for (size_t s = 0; s < P; s++) {
            if (K == 0) {
                cxI[s] = a1[s]; cyI[s] = b1[s]; xI[s] = c1[s]; yI[s] = d1[s];
            } else {
                cxI[s] = 0.5 * (a0[s] + a1[s]); cyI[s] = 0.5 * (b0[s] + b1[s]);
                xI[s] = 0.5 * (c0[s] + c1[s]); yI[s] = 0.5 * (d0[s] + d1[s]);
            }
        }
        double *z = zh + (size_t)K * P;
        og_view_scalar(g, z, ST_C, MODE_X, 0, qx);
        og_view_scalar(g, z, ST_C, MODE_Y, 0, qy);
        o_fv_tp_2d(g, t, z, qx, qy, cxI, cyI, xI, yI, NULL, NULL, ZX, ZY);
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                size_t c = IX(g, i, j), e = IX(g, i + 1, j), nn = IX(g, i, j + 1);
                zn[(size_t)K * P + c] = (z[c] * area[c] + ZX[c] - ZX[e] + ZY[c] - ZY[nn]) /
                                        (area[c] + xI[c] - xI[e] + yI[c] - yI[nn]);
            }
    }
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            size_t c = IX(g, i, j);
            zn[(size_t)nz * P + c] = zs[c];
            for (int k = 0; k < nz; k++)
                PL(delz, t, k, nz)[c] = zn[(size_t)(k + 1) * P + c] - zn[(size_t)k * P + c];
        }
    free(zh); free(zn); free(qx); free(qy); free(ZX); free(ZY); free(cxI); free(cyI);
    free(xI); free(yI);
}

/* ----------------------------------------------------------- nh_p_grad */
/*
 * Values at cell corners by the fourth-order (-1,7,7,-1)/12 tensor
 * interpolation (inner pass along x reading the x-sweep corner view), or the
 * mean of the three cells at a cube vertex; the finite-volume pressure
 * gradient between the two corners of each D-grid edge updates u and v.
 */
static void corner_interp(const OGrid *g, const double *q, double *qB)
{
    int n = g->n;
    size_t P = o_plane(g);
    double *qx = dalloc(P);
    /* one-sided stencils at tile edges (option edge_interp, cube): the pass
     * along x on rows inside the tile, the pass along y on every corner
     * column (all lie on or inside the tile) */
    const int ei = g->edge_interp && g->kind == 1;
    og_view_scalar(g, q, ST_C, MODE_X, 0, qx);
    for (int j = 0; j <= n; j++)
        for (int i = 0; i <= n; i++) {
            if (og_is_vertex(g, i, j)) {
                double s = 0.0;
                int cells[4][2] = {{i - 1, j - 1}, {i, j - 1}, {i, j}, {i - 1, j}};
                for (int c = 0; c < 4; c++) {
                    if (og_region(g, ST_C, cells[c][0], cells[c][1]) == 2) continue;
                    s += q[IX(g, cells[c][0], cells[c][1])];
                }
                qB[IX(g, i, j)] = s / 3.0;
                continue;
            }
            /* inner pass along x on the rows j - 2 .. j + 1, then along y */
            double rows[4];
            for (int b = 0; b < 4; b++) {
                int r = j + b - 2;
                rows[b] = o_interp(OI_FACE_MEAN, qx + IX(g, 0, r), 1, 0, i, n, ei && r >= 0 && r < n);
            }
            qB[IX(g, i, j)] = o_interp(OI_FACE_MEAN, rows, 1, j - 2, j, n, ei);
        }
    free(qx);
}

/* c_sw's corner vorticity of one level of every tile from C-grid winds */
void o_corner_vort_all(const OGrid *g, const double *uc, const double *vc, double *out)
{
    size_t P = o_plane(g);
    for (int t = 0; t < g->T; t++)
        for (int j = 0; j <= g->n; j++)
            for (int i = 0; i <= g->n; i++)
                out[(size_t)t * P + IX(g, i, j)] = o_corner_vort(g, t, uc + (size_t)t * P, vc + (size_t)t * P, i, j);
}

/* corner values of one level of every tile (halos already filled) */
void o_corner_values(const OGrid *g, const double *q, double *qB)
{
    size_t P = o_plane(g);
    for (int t = 0; t < g->T; t++) corner_interp(g, q + (size_t)t * P, qB + (size_t)t * P);
}

static void nhpgrad_tile(const OGrid *g, int t, double bdt, double *u, double *v,
                         const double *delp, const double *pfull, const double *phi)
{
    int n = g->n, nz = g->nz;
    size_t P = o_plane(g), o = (size_t)t * P;
    double *pB = dalloc((size_t)(nz + 1) * P), *zB = dalloc((size_t)(nz + 1) * P),
           *dB = dalloc(P);
    for (int K = 0; K <= nz; K++) {
        corner_interp(g, PL(pfull, t, K, nz + 1), pB + (size_t)K * P);
        corner_interp(g, PL(phi, t, K, nz + 1), zB + (size_t)K * P);
    }
    for (int k = 0; k < nz; k++) {
        corner_interp(g, PL(delp, t, k, nz), dB);
        const double *p0 = pB + (size_t)k * P, *p1 = pB + (size_t)(k + 1) * P;
        const double *z0 = zB + (size_t)k * P, *z1 = zB + (size_t)(k + 1) * P;
        double *U = PL(u, t, k, nz), *V = PL(v, t, k, nz);
        for (int j = 0; j <= n; j++)
            for (int i = 0; i < n; i++) {
                size_t f = IX(g, i, j), W = IX(g, i, j), E = IX(g, i + 1, j);
                U[f] += o_pgf(bdt, g->dx[o + f], dB[W], dB[E], z0[W], z1[W], z0[E], z1[E],
                              p0[W], p1[W], p0[E], p1[E]);
            }
        for (int j = 0; j < n; j++)
            for (int i = 0; i <= n; i++) {
                size_t f = IX(g, i, j), W = IX(g, i, j), E = IX(g, i, j + 1);
                V[f] += o_pgf(bdt, g->dy[o + f], dB[W], dB[E], z0[W], z1[W], z0[E], z1[E],
                              p0[W], p1[W], p0[E], p1[E]);
            }
    }
    free(pB); free(zB); free(dB);
}

/* ------------------------------------------------------- substep driver */

static int all_finite(const OGrid *g, const double *f, int nlev)
{
    size_t P = o_plane(g);
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nlev; k++)
            for (int j = 0; j < g->n; j++)
                for (int i = 0; i < g->n; i++)
                    if (!isfinite(f[((size_t)t * nlev + k) * P + IX(g, i, j)])) return 0;
    return 1;
}

/* status codes shared in meaning (not in code) with the library */
#define ORC_OK 0
#define ORC_ECFL (-6)
#define ORC_ENONFINITE (-7)

int orc_substeps_impl(const OGrid *g, OState *s, double dt, int n_split, int stop_stage,
                      double **dbg)
{
    int T = g->T, nz = g->nz;
    size_t P = o_plane(g), F3 = (size_t)T * nz * P, F3i = (size_t)T * (nz + 1) * P;
    double bdt = dt / n_split, dt2 = 0.5 * bdt;
    double *delpc = dalloc(F3), *ptc = dalloc(F3), *wc = dalloc(F3), *ax = dalloc(F3),
           *ay = dalloc(F3), *crx = dalloc(F3), *cry = dalloc(F3), *xfx = dalloc(F3),
           *yfx = dalloc(F3), *pkc = dalloc(F3i), *gz = dalloc(F3i);
    double *zs = dalloc((size_t)T * P);
    /* debug outputs of the last substep: c_sw's corner and d_sw's cell
     * absolute vorticity (each substep overwrites them) */
    double *vortc = dbg ? dbg[11] : NULL, *vortd = dbg ? dbg[12] : NULL;
    int cfl = 0, status = ORC_OK;
    double *hd = NULL, *hd2 = NULL;
    if (g->nord > 0 && g->d4_bg > 0.0) {
        hd = dalloc(F3);
        hd2 = dalloc(F3);
    }
    double *efb[6] = {0, 0, 0, 0, 0, 0}, **ef = NULL;
    if (g->edge_fix && g->kind == 1) {
        for (int q = 0; q < 6; q++) efb[q] = dalloc(F3);
        ef = efb;
    }

    for (size_t q = 0; q < (size_t)T * P; q++) zs[q] = s->phis ? s->phis[q] / O_GRAV : 0.0;
    og_fill_scalar(g, zs, 1, ST_C, 0);
    /* humidity is constant over the call: its halo once */
    if (s->qv) og_fill_scalar(g, s->qv, nz, ST_C, 0);
    /* accumulators restart with every call; delp at entry is kept */
    memset(s->mfx, 0, F3 * sizeof(double));
    memset(s->mfy, 0, F3 * sizeof(double));
    memset(s->cx, 0, F3 * sizeof(double));
    memset(s->cy, 0, F3 * sizeof(double));
    memcpy(s->dp0, s->delp, F3 * sizeof(double));

    for (int it = 0; it < n_split; it++) {
        int last = (it == n_split - 1);
#define STOP(st) if (last && stop_stage == (st)) goto done
        og_fill_pair(g, s->u, ST_Y, s->v, ST_X, nz, PAIR_SIGNED);
        og_fill_scalar(g, s->delp, nz, ST_C, 0);
        og_fill_scalar(g, s->pt, nz, ST_C, 0);
        og_fill_scalar(g, s->w, nz, ST_C, 0);
        og_fill_scalar(g, s->delz, nz, ST_C, 0);
        STOP(1);
#pragma omp parallel for collapse(2) schedule(dynamic)
        for (int t = 0; t < T; t++)
            for (int k = 0; k < nz; k++)
                c_sw_plane(g, t, dt2, PL(s->u, t, k, nz), PL(s->v, t, k, nz),
                           PL(s->delp, t, k, nz), PL(s->pt, t, k, nz), PL(s->w, t, k, nz),
                           PL(s->uc, t, k, nz), PL(s->vc, t, k, nz), PL(delpc, t, k, nz),
                           PL(ptc, t, k, nz), PL(wc, t, k, nz), PL(ax, t, k, nz),
                           PL(ay, t, k, nz), vortc ? PL(vortc, t, k, nz) : NULL);
        STOP(2);
#pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < T; t++)
            dzc_riemc_tile(g, t, dt2, s->delz, zs + (size_t)t * P, ax, ay, delpc, ptc, wc, s->qv, pkc, gz);
        STOP(3);
#pragma omp parallel for collapse(2) schedule(dynamic)
        for (int t = 0; t < T; t++)
            for (int k = 0; k < nz; k++) pgradc_plane(g, t, k, dt2, delpc, pkc, gz, s->uc, s->vc);
        STOP(4);
        og_fill_pair(g, s->uc, ST_X, s->vc, ST_Y, nz, PAIR_SIGNED);
        STOP(5);
        if (hd) {
            /* corner divergence of the D-grid winds, then nord corner
             * Laplacians, each after a fill of the corner halo */
#pragma omp parallel for collapse(2)
            for (int t = 0; t < T; t++)
                for (int k = 0; k < nz; k++)
                    o_corner_div(g, t, PL(s->u, t, k, nz), PL(s->v, t, k, nz), PL(hd, t, k, nz));
            for (int r = 0; r < g->nord; r++) {
                og_fill_scalar(g, hd, nz, ST_B, 0);
#pragma omp parallel for collapse(2)
                for (int t = 0; t < T; t++)
                    for (int k = 0; k < nz; k++) o_corner_lap(g, t, PL(hd, t, k, nz), PL(hd2, t, k, nz));
                double *sw = hd; hd = hd2; hd2 = sw;
            }
        }
#pragma omp parallel for collapse(2) schedule(dynamic) reduction(| : cfl)
        for (int t = 0; t < T; t++)
            for (int k = 0; k < nz; k++) {
                int c = 0;
                double *efp[6];
                for (int q = 0; q < 6; q++) efp[q] = ef ? PL(ef[q], t, k, nz) : NULL;
                d_sw_plane(g, t, k, bdt, PL(s->u, t, k, nz), PL(s->v, t, k, nz),
                           PL(s->uc, t, k, nz), PL(s->vc, t, k, nz), PL(s->delp, t, k, nz),
                           PL(s->pt, t, k, nz), PL(s->w, t, k, nz), PL(s->mfx, t, k, nz),
                           PL(s->mfy, t, k, nz), PL(s->cx, t, k, nz), PL(s->cy, t, k, nz),
                           PL(crx, t, k, nz), PL(cry, t, k, nz), PL(xfx, t, k, nz),
                           PL(yfx, t, k, nz), hd ? PL(hd, t, k, nz) : NULL, ef ? efp : NULL, &c,
                           vortd ? PL(vortd, t, k, nz) : NULL);
                cfl |= c;
            }
        if (ef)
            o_edge_fix_dsw(g, ef[0], ef[1], ef[2], ef[3], ef[4], ef[5], s->delp, s->pt, s->w, s->mfx, s->mfy);
        STOP(6);
#pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < T; t++)
            dzd_tile(g, t, s->delz, zs + (size_t)t * P, crx, cry, xfx, yfx);
        STOP(7);
#pragma omp parallel for collapse(2) schedule(dynamic)
        for (int t = 0; t < T; t++)
            for (int j = 0; j < g->n; j++) {
                double *cd = dalloc(nz), *ct = dalloc(nz), *cz = dalloc(nz), *cw = dalloc(nz);
                double *wo = dalloc(nz), *dzo = dalloc(nz), *pf = dalloc(nz + 1), *ph = dalloc(nz + 1);
                for (int i = 0; i < g->n; i++) {
                    size_t c = IX(g, i, j);
                    for (int k = 0; k < nz; k++) {
                        cd[k] = PL(s->delp, t, k, nz)[c];
                        ct[k] = PL(s->pt, t, k, nz)[c] * o_virt(s->qv, (size_t)(t * nz + k) * P + c);
                        cz[k] = PL(s->delz, t, k, nz)[c];
                        cw[k] = PL(s->w, t, k, nz)[c];
                    }
                    o_sim1b(nz, bdt, g->beta, g->pp_order, g->ptop, zs[(size_t)t * P + c], cd, ct, cz, cw, wo, dzo, pf,
                            ph, 0, 0);
                    for (int k = 0; k < nz; k++) {
                        PL(s->w, t, k, nz)[c] = wo[k];
                        PL(s->delz, t, k, nz)[c] = dzo[k];
                    }
                    for (int K = 0; K <= nz; K++) {
                        PL(s->pfull, t, K, nz + 1)[c] = pf[K];
                        PL(s->phi, t, K, nz + 1)[c] = ph[K];
                    }
                }
                free(cd); free(ct); free(cz); free(cw); free(wo); free(dzo); free(pf); free(ph);
            }
        STOP(8);
        og_fill_scalar(g, s->pfull, nz + 1, ST_C, 0);
        og_fill_scalar(g, s->phi, nz + 1, ST_C, 0);
        og_fill_scalar(g, s->delp, nz, ST_C, 0);
        STOP(9);
#pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < T; t++) nhpgrad_tile(g, t, bdt, s->u, s->v, s->delp, s->pfull, s->phi);
#undef STOP
    }
done:
    free(hd);
    free(hd2);
    for (int q = 0; q < 6; q++) free(efb[q]);
    if (dbg) {
        double *src[] = {delpc, ptc, wc, ax, ay, crx, cry, xfx, yfx};
        for (int q = 0; q < 9; q++)
            if (dbg[q]) memcpy(dbg[q], src[q], F3 * sizeof(double));
        if (dbg[9]) memcpy(dbg[9], pkc, F3i * sizeof(double));
        if (dbg[10]) memcpy(dbg[10], gz, F3i * sizeof(double));
    }
    if (cfl) status = ORC_ECFL;
    else {
        double *chk[] = {s->u, s->v, s->w, s->delp, s->pt, s->delz};
        for (int q = 0; q < 6; q++)
            if (!all_finite(g, chk[q], nz)) status = ORC_ENONFINITE;
    }
    free(delpc); free(ptc); free(wc); free(ax); free(ay); free(crx); free(cry); free(xfx);
    free(yfx); free(pkc); free(gz); free(zs);
    return status;
}

/* ------------------------------------------------------ tracer transport */
/*
 * Tracer advection of the remapping step with the fluxes accumulated over
 * the acoustic substeps: area fluxes rebuilt from the accumulated Courant
 * numbers, a sub-cycle count that keeps every sub-cycle Courant number at
 * most 1, and per sub-cycle a mass-weighted flux-form update in which the
 * layer mass advances with the accumulated mass fluxes.
 */
int orc_tracer_impl(const OGrid *g, double **q, int nq, const double *dp0, const double *mfx,
                    const double *mfy, const double *cx_in, const double *cy_in, int nsplt,
                    int *nsplt_used)
{
    int T = g->T, nz = g->nz, n = g->n;
    size_t P = o_plane(g), F3 = (size_t)T * nz * P;
    double *cx = dalloc(F3), *cy = dalloc(F3);
    memcpy(cx, cx_in, F3 * sizeof(double));
    memcpy(cy, cy_in, F3 * sizeof(double));
    og_fill_pair(g, cx, ST_X, cy, ST_Y, nz, PAIR_SIGNED);
    if (nsplt <= 0) {
        double cmax = 0.0;
        for (int t = 0; t < T; t++)
            for (int k = 0; k < nz; k++) {
                for (int j = 0; j < n; j++)
                    for (int i = 0; i <= n; i++) {
                        double a = fabs(PL(cx, t, k, nz)[IX(g, i, j)]);
                        if (a > cmax) cmax = a;
                    }
                for (int j = 0; j <= n; j++)
                    for (int i = 0; i < n; i++) {
                        double a = fabs(PL(cy, t, k, nz)[IX(g, i, j)]);
                        if (a > cmax) cmax = a;
                    }
            }
        nsplt = (int)ceil(cmax);
        if (nsplt < 1) nsplt = 1;
    }
    if (nsplt_used) *nsplt_used = nsplt;
    double rs = (double)nsplt;
    double *xfx = dalloc(F3), *yfx = dalloc(F3), *dp1 = dalloc(F3), *dp2 = dalloc(F3);
    double *crs = dalloc(F3), *crys = dalloc(F3), *mxs = dalloc(F3), *mys = dalloc(F3);
    double *efx = NULL, *efy = NULL;
    if (g->edge_fix && g->kind == 1) {
        efx = dalloc(F3);
        efy = dalloc(F3);
    }
    memcpy(dp1, dp0, F3 * sizeof(double));
#pragma omp parallel for collapse(2)
    for (int t = 0; t < T; t++)
        for (int k = 0; k < nz; k++) {
            size_t o = (size_t)t * P;
            double *dxaX = dalloc(P), *dyaX = dalloc(P), *dxaY = dalloc(P), *dyaY = dalloc(P);
            og_view_pair(g, g->dxa + o, ST_C, g->dya + o, ST_C, MODE_X, PAIR_ABS, dxaX, dyaX);
            og_view_pair(g, g->dxa + o, ST_C, g->dya + o, ST_C, MODE_Y, PAIR_ABS, dxaY, dyaY);
            const double *CX = PL(cx, t, k, nz), *CY = PL(cy, t, k, nz);
            double *XF = PL(xfx, t, k, nz), *YF = PL(yfx, t, k, nz);
            for (int j = -3; j <= n + 2; j++)
                for (int i = 0; i <= n; i++) {
                    size_t f = IX(g, i, j), up = CX[f] > 0.0 ? IX(g, i - 1, j) : f;
                    XF[f] = CX[f] * dxaX[up] * g->dy[o + f] * g->sin_u[o + f];
                }
            for (int j = 0; j <= n; j++)
                for (int i = -3; i <= n + 2; i++) {
                    size_t f = IX(g, i, j), up = CY[f] > 0.0 ? IX(g, i, j - 1) : f;
                    YF[f] = CY[f] * dyaY[up] * g->dx[o + f] * g->sin_v[o + f];
                }
            free(dxaX); free(dyaX); free(dxaY); free(dyaY);
        }
    for (size_t s = 0; s < F3; s++) {
        crs[s] = cx[s] / rs; crys[s] = cy[s] / rs;
        xfx[s] = xfx[s] / rs; yfx[s] = yfx[s] / rs;
        mxs[s] = mfx[s] / rs; mys[s] = mfy[s] / rs;
    }
    for (int it = 0; it < nsplt; it++) {
#pragma omp parallel for collapse(2)
        for (int t = 0; t < T; t++)
            for (int k = 0; k < nz; k++) {
                size_t o = (size_t)t * P;
                const double *d1 = PL(dp1, t, k, nz), *MX = PL(mxs, t, k, nz), *MY = PL(mys, t, k, nz);
                double *d2 = PL(dp2, t, k, nz);
                for (int j = 0; j < n; j++)
                    for (int i = 0; i < n; i++) {
                        size_t c = IX(g, i, j);
                        d2[c] = d1[c] + (MX[c] - MX[IX(g, i + 1, j)] + MY[c] - MY[IX(g, i, j + 1)]) /
                                            g->area[o + c];
                    }
            }
        for (int m = 0; m < nq; m++) {
            og_fill_scalar(g, q[m], nz, ST_C, 0);
#pragma omp parallel for collapse(2)
            for (int t = 0; t < T; t++)
                for (int k = 0; k < nz; k++) {
                    size_t o = (size_t)t * P;
                    double *Q = PL(q[m], t, k, nz);
                    double *qx = dalloc(P), *qy = dalloc(P), *FX = dalloc(P), *FY = dalloc(P);
                    double *keepX = efx ? PL(efx, t, k, nz) : NULL, *keepY = efy ? PL(efy, t, k, nz) : NULL;
                    og_view_scalar(g, Q, ST_C, MODE_X, 0, qx);
                    og_view_scalar(g, Q, ST_C, MODE_Y, 0, qy);
                    o_fv_tp_2d_ord(g, g->hord_tr ? g->hord_tr : g->hord, t, Q, qx, qy, PL(crs, t, k, nz), PL(crys, t, k, nz),
                               PL(xfx, t, k, nz), PL(yfx, t, k, nz), PL(mxs, t, k, nz),
                               PL(mys, t, k, nz), FX, FY);
                    const double *d1 = PL(dp1, t, k, nz), *d2 = PL(dp2, t, k, nz);
                    for (int j = 0; j < n; j++)
                        for (int i = 0; i < n; i++) {
                            size_t c = IX(g, i, j);
                            double a = g->area[o + c];
                            Q[c] = (Q[c] * d1[c] * a + FX[c] - FX[IX(g, i + 1, j)] + FY[c] -
                                    FY[IX(g, i, j + 1)]) / (d2[c] * a);
                        }
                    if (keepX) {
                        memcpy(keepX, FX, P * sizeof(double));
                        memcpy(keepY, FY, P * sizeof(double));
                    }
                    free(qx); free(qy); free(FX); free(FY);
                }
            if (efx) o_edge_fix_tracer(g, efx, efy, dp2, q[m]);
        }
        double *tmp = dp1; dp1 = dp2; dp2 = tmp;
    }
    free(cx); free(cy); free(xfx); free(yfx); free(dp1); free(dp2); free(crs); free(crys);
    free(mxs); free(mys); free(efx); free(efy);
    return 0;
}

/* ---------------------------------------------------- compensated sums */
/* Neumaier summation in the fixed order (tile, level, row, column). */
typedef struct { double s, c; } Neu;
static void neu_add(Neu *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* out[0] = sum delp*area, out[1] = sum pt*delp*area, out[2+m] = sum q_m*delp*area */
void orc_mass_sums_impl(const OGrid *g, const double *delp, const double *pt,
                        const double *const *q, int nq, double *out)
{
    int T = g->T, nz = g->nz, n = g->n;
    size_t P = o_plane(g);
    for (int m = -2; m < nq; m++) {
        Neu a = {0.0, 0.0};
        for (int t = 0; t < T; t++)
            for (int k = 0; k < nz; k++)
                for (int j = 0; j < n; j++)
                    for (int i = 0; i < n; i++) {
                        size_t c = IX(g, i, j), s = ((size_t)t * nz + k) * P + c;
                        double mass = delp[s] * g->area[(size_t)t * P + c];
                        double x = m == -2 ? mass : (m == -1 ? pt[s] * mass : q[m][s] * mass);
                        neu_add(&a, x);
                    }
        out[m + 2] = a.s + a.c;
    }
}
