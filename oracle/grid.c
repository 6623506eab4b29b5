/*
 * ORACLE (test infrastructure only): grids and metric terms.
 *
 * The paper runs FV3 on the gnomonic cubed sphere (Sec. II).  The oracle
 * builds the equiangular gnomonic grid: face t has a right-handed frame
 * (c, e1, e2) and corner (I,J) is the normalised point
 * c + tan(a_I) e1 + tan(b_J) e2 with a_I = (2I - n) pi / (4n).  Connectivity
 * between tiles is found by matching shared edge end points, which fixes the
 * lattice rotation used for the orientation transform of vector halos.
 * Lengths are great-circle arcs, areas spherical excesses (sum of the excesses
 * of a triangle fan), Coriolis f = 2 Omega sin(latitude).  Faces on a tile edge
 * carry cos = 0, sin = 1 so that the normal wind there is the stored wind, the
 * tile-edge region rule printed in Sec. V-B.
 *
 * The doubly periodic grid is the single-tile test fixture: every length is
 * delta, every area delta^2, sin = 1, cos = 0, f = f0.
 */
#include "orc.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* frame (c, e1, e2) of each cube face; e1 x e2 = c */
static const double FRAME[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {-1, 0, 0}, {0, -1, 0}},
    {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double *a)
{
    double r = sqrt(dot3(a, a));
    a[0] /= r; a[1] /= r; a[2] /= r;
}
/* great-circle angle between two unit vectors */
static double arc(const double *a, const double *b)
{
    double c[3];
    cross3(a, b, c);
    return atan2(sqrt(dot3(c, c)), dot3(a, b));
}
/* unit tangent at p pointing along the chord d */
static void tangent(const double *p, const double *d, double *out)
{
    double s = dot3(d, p);
    out[0] = d[0] - s * p[0]; out[1] = d[1] - s * p[1]; out[2] = d[2] - s * p[2];
    normalize3(out);
}
/* Spherical excess of the triangle (a, b, c) on the unit sphere, from the
 * Van Oosterom-Strackee relation tan(E/2) = |a.(b x c)| / (1 + a.b + b.c + c.a),
 * which keeps full relative precision for small triangles. */
static double tri_excess(const double *a, const double *b, const double *c)
{
    double bc[3];
    cross3(b, c, bc);
    return 2.0 * atan2(fabs(dot3(a, bc)), 1.0 + dot3(a, b) + dot3(b, c) + dot3(c, a));
}
/* excess of a convex spherical polygon, fanned from its first vertex */
static double excess(const double *const *v, int m)
{
    double s = 0;
    for (int k = 1; k + 1 < m; k++) s += tri_excess(v[0], v[k], v[k + 1]);
    return s;
}

static void gnomonic(int t, int n, int I, int J, double *out)
{
    double ta = (I == 0) ? -1.0 : (I == n ? 1.0 : tan((2 * I - n) * M_PI / (4.0 * n)));
    double tb = (J == 0) ? -1.0 : (J == n ? 1.0 : tan((2 * J - n) * M_PI / (4.0 * n)));
    for (int d = 0; d < 3; d++) out[d] = FRAME[t][0][d] + ta * FRAME[t][1][d] + tb * FRAME[t][2][d];
    normalize3(out);
}

static double *zalloc(size_t n) { return (double *)calloc(n, sizeof(double)); }

static int connect(OGrid *g, char *err, size_t errlen)
{
    int n = g->n;
    int ends[4][2][2] = {{{0, 0}, {0, n}}, {{n, 0}, {n, n}}, {{0, 0}, {n, 0}}, {{0, n}, {n, n}}};
    int inward[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    int rots[4][2][2] = {{{1, 0}, {0, 1}}, {{0, -1}, {1, 0}}, {{-1, 0}, {0, -1}}, {{0, 1}, {-1, 0}}};
    double tol = 1e-12;
    for (int t = 0; t < 6; t++)
        for (int e = 0; e < 4; e++) {
            double a0[3], a1[3];
            gnomonic(t, n, ends[e][0][0], ends[e][0][1], a0);
            gnomonic(t, n, ends[e][1][0], ends[e][1][1], a1);
            int found = 0;
            for (int tb = 0; tb < 6 && !found; tb++) {
                if (tb == t) continue;
                for (int eb = 0; eb < 4 && !found; eb++)
                    for (int o = 0; o < 2 && !found; o++) {
                        double b0[3], b1[3];
                        int *Q0 = ends[eb][o], *Q1 = ends[eb][1 - o];
                        gnomonic(tb, n, Q0[0], Q0[1], b0);
                        gnomonic(tb, n, Q1[0], Q1[1], b1);
                        if (arc(a0, b0) > tol || arc(a1, b1) > tol) continue;
                        int tA[2] = {(ends[e][1][0] - ends[e][0][0]) / n, (ends[e][1][1] - ends[e][0][1]) / n};
                        int tB[2] = {(Q1[0] - Q0[0]) / n, (Q1[1] - Q0[1]) / n};
                        int r;
                        for (r = 0; r < 4; r++) {
                            int *m0 = rots[r][0], *m1 = rots[r][1];
                            if (m0[0] * tA[0] + m0[1] * tA[1] == tB[0] && m1[0] * tA[0] + m1[1] * tA[1] == tB[1]) break;
                        }
                        if (r == 4) continue;
                        /* our outward normal must become the neighbour's inward normal */
                        int on[2] = {-inward[e][0], -inward[e][1]};
                        int mapped[2] = {rots[r][0][0] * on[0] + rots[r][0][1] * on[1],
                                         rots[r][1][0] * on[0] + rots[r][1][1] * on[1]};
                        if (mapped[0] != inward[eb][0] || mapped[1] != inward[eb][1]) {
                            snprintf(err, errlen, "tile %d edge %d: orientation mismatch", t, e);
                            return -1;
                        }
                        g->nbr[t][e] = tb;
                        memcpy(g->R[t][e], rots[r], sizeof(int) * 4);
                        g->P0[t][e][0] = ends[e][0][0]; g->P0[t][e][1] = ends[e][0][1];
                        g->Q0[t][e][0] = Q0[0]; g->Q0[t][e][1] = Q0[1];
                        found = 1;
                    }
            }
            if (!found) {
                snprintf(err, errlen, "tile %d edge %d: no neighbour found", t, e);
                return -1;
            }
        }
    return 0;
}

#define ALLOC_METRICS(g, P)                                                                    \
    do {                                                                                       \
        double **m[] = {&g->dx, &g->dy, &g->dxc, &g->dyc, &g->dxa, &g->dya, &g->area,         \
                        &g->area_c, &g->fC, &g->fB, &g->sin_u, &g->cos_u, &g->sin_v,          \
                        &g->cos_v, &g->sin_a, &g->cos_a};                                      \
        for (size_t q = 0; q < sizeof(m) / sizeof(m[0]); q++) *m[q] = zalloc(P);               \
    } while (0)

static void periodic_metrics(OGrid *g)
{
    size_t P = (size_t)g->T * o_plane(g);
    double d = g->delta;
    for (size_t s = 0; s < P; s++) {
        g->dx[s] = g->dy[s] = g->dxc[s] = g->dyc[s] = g->dxa[s] = g->dya[s] = d;
        g->area[s] = g->area_c[s] = d * d;
        g->fC[s] = g->fB[s] = g->f0;
        g->sin_u[s] = g->sin_v[s] = g->sin_a[s] = 1.0;
        g->cos_u[s] = g->cos_v[s] = g->cos_a[s] = 0.0;
    }
}

static void cube_metrics(OGrid *g)
{
    int n = g->n;
    size_t P = o_plane(g);
    double a = g->radius, a2 = a * a;
    for (int d = 0; d < 3; d++) {
        g->cpos[d] = zalloc(6 * P);
        g->bpos[d] = zalloc(6 * P);
    }
#define BP(t, i, j, out) do { for (int d_ = 0; d_ < 3; d_++) (out)[d_] = g->bpos[d_][(t) * P + IX(g, i, j)]; } while (0)
#define CP(t, i, j, out) do { for (int d_ = 0; d_ < 3; d_++) (out)[d_] = g->cpos[d_][(t) * P + IX(g, i, j)]; } while (0)
    for (int t = 0; t < 6; t++) {
        for (int J = 0; J <= n; J++)
            for (int I = 0; I <= n; I++) {
                double p[3];
                gnomonic(t, n, I, J, p);
                for (int d = 0; d < 3; d++) g->bpos[d][t * P + IX(g, I, J)] = p[d];
            }
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double c[3] = {0, 0, 0}, p[3];
                int ci[4][2] = {{i, j}, {i + 1, j}, {i + 1, j + 1}, {i, j + 1}};
                for (int q = 0; q < 4; q++) {
                    BP(t, ci[q][0], ci[q][1], p);
                    for (int d = 0; d < 3; d++) c[d] += p[d];
                }
                normalize3(c);
                for (int d = 0; d < 3; d++) g->cpos[d][t * P + IX(g, i, j)] = c[d];
            }
    }
    for (int d = 0; d < 3; d++) og_fill_scalar(g, g->cpos[d], 1, ST_C, 0);

    for (int t = 0; t < 6; t++) {
        size_t o = (size_t)t * P;
        /* x-faces */
        for (int j = 0; j < n; j++)
            for (int i = 0; i <= n; i++) {
                double b0[3], b1[3], cw[3], ce[3], m[3], ex[3], ey[3], d1[3], d2[3];
                BP(t, i, j, b0); BP(t, i, j + 1, b1);
                CP(t, i - 1, j, cw); CP(t, i, j, ce);
                for (int d = 0; d < 3; d++) { m[d] = b0[d] + b1[d]; d1[d] = b1[d] - b0[d]; d2[d] = ce[d] - cw[d]; }
                normalize3(m);
                g->dy[o + IX(g, i, j)] = a * arc(b0, b1);
                g->dxc[o + IX(g, i, j)] = a * arc(cw, ce);
                tangent(m, d1, ey);
                tangent(m, d2, ex);
                double cs = dot3(ex, ey);
                if (i == 0 || i == n) cs = 0.0;
                g->cos_u[o + IX(g, i, j)] = cs;
                g->sin_u[o + IX(g, i, j)] = (i == 0 || i == n) ? 1.0 : sqrt(1.0 - cs * cs);
            }
        /* y-faces */
        for (int j = 0; j <= n; j++)
            for (int i = 0; i < n; i++) {
                double b0[3], b1[3], cs_[3], cn[3], m[3], ex[3], ey[3], d1[3], d2[3];
                BP(t, i, j, b0); BP(t, i + 1, j, b1);
                CP(t, i, j - 1, cs_); CP(t, i, j, cn);
                for (int d = 0; d < 3; d++) { m[d] = b0[d] + b1[d]; d1[d] = b1[d] - b0[d]; d2[d] = cn[d] - cs_[d]; }
                normalize3(m);
                g->dx[o + IX(g, i, j)] = a * arc(b0, b1);
                g->dyc[o + IX(g, i, j)] = a * arc(cs_, cn);
                tangent(m, d1, ex);
                tangent(m, d2, ey);
                double cs = dot3(ex, ey);
                if (j == 0 || j == n) cs = 0.0;
                g->cos_v[o + IX(g, i, j)] = cs;
                g->sin_v[o + IX(g, i, j)] = (j == 0 || j == n) ? 1.0 : sqrt(1.0 - cs * cs);
            }
        /* cells */
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double b[4][3], c[3], mw[3], me[3], ms[3], mn[3], dxv[3], dyv[3], ex[3], ey[3];
                BP(t, i, j, b[0]); BP(t, i + 1, j, b[1]); BP(t, i + 1, j + 1, b[2]); BP(t, i, j + 1, b[3]);
                CP(t, i, j, c);
                for (int d = 0; d < 3; d++) {
                    mw[d] = b[0][d] + b[3][d]; me[d] = b[1][d] + b[2][d];
                    ms[d] = b[0][d] + b[1][d]; mn[d] = b[3][d] + b[2][d];
                }
                normalize3(mw); normalize3(me); normalize3(ms); normalize3(mn);
                const double *v[4] = {b[0], b[1], b[2], b[3]};
                g->area[o + IX(g, i, j)] = a2 * excess(v, 4);
                g->dxa[o + IX(g, i, j)] = a * arc(mw, me);
                g->dya[o + IX(g, i, j)] = a * arc(ms, mn);
                g->fC[o + IX(g, i, j)] = 2.0 * g->omega * c[2];
                for (int d = 0; d < 3; d++) { dxv[d] = me[d] - mw[d]; dyv[d] = mn[d] - ms[d]; }
                tangent(c, dxv, ex);
                tangent(c, dyv, ey);
                double cs = dot3(ex, ey);
                g->cos_a[o + IX(g, i, j)] = cs;
                g->sin_a[o + IX(g, i, j)] = sqrt(1.0 - cs * cs);
            }
        /* corners: dual-cell area from the surrounding centres (3 at a cube vertex) */
        for (int j = 0; j <= n; j++)
            for (int i = 0; i <= n; i++) {
                double c00[3], c10[3], c11[3], c01[3], b[3];
                CP(t, i - 1, j - 1, c00); CP(t, i, j - 1, c10); CP(t, i, j, c11); CP(t, i - 1, j, c01);
                BP(t, i, j, b);
                g->fB[o + IX(g, i, j)] = 2.0 * g->omega * b[2];
                if (og_is_vertex(g, i, j)) {
                    const double *v[3];
                    int m = 0;
                    /* skip the centre that would lie in the missing corner block */
                    if (!(i == 0 && j == 0)) v[m++] = c00;
                    if (!(i == n && j == 0)) v[m++] = c10;
                    if (!(i == n && j == n)) v[m++] = c11;
                    if (!(i == 0 && j == n)) v[m++] = c01;
                    g->area_c[o + IX(g, i, j)] = a2 * excess(v, 3);
                } else {
                    const double *v[4] = {c00, c10, c11, c01};
                    g->area_c[o + IX(g, i, j)] = a2 * excess(v, 4);
                }
            }
    }
#undef BP
#undef CP
    og_fill_pair(g, g->dx, ST_Y, g->dy, ST_X, 1, PAIR_ABS);
    og_fill_pair(g, g->dxc, ST_X, g->dyc, ST_Y, 1, PAIR_ABS);
    og_fill_pair(g, g->sin_u, ST_X, g->sin_v, ST_Y, 1, PAIR_ABS);
    og_fill_pair(g, g->cos_u, ST_X, g->cos_v, ST_Y, 1, PAIR_COS);
    og_fill_pair(g, g->dxa, ST_C, g->dya, ST_C, 1, PAIR_ABS);
    og_fill_scalar(g, g->area, 1, ST_C, 0);
    og_fill_scalar(g, g->fC, 1, ST_C, 0);
    og_fill_scalar(g, g->sin_a, 1, ST_C, 0);
    og_fill_scalar(g, g->cos_a, 1, ST_C, 1);
}

OGrid *og_new(int kind, int n, int nz, double delta, double f0, double radius, double omega,
              double ptop, char *err, size_t errlen)
{
    if (n < 4 || nz < 1 || (kind != 0 && kind != 1)) {
        snprintf(err, errlen, "bad grid size or kind");
        return NULL;
    }
    OGrid *g = (OGrid *)calloc(1, sizeof(OGrid));
    g->kind = kind; g->n = n; g->nz = nz; g->T = kind == 1 ? 6 : 1; g->N = n + 2 * H + 1;
    g->delta = delta; g->f0 = f0; g->radius = radius; g->omega = omega; g->ptop = ptop;
    g->beta = 1.0;
    g->hord = 8;
    g->hord_tr = 0;
    g->pp_order = 2;
    g->nord = 0;
    g->d4_bg = 0.0;
    g->vtdm = 0.0;
    g->edge_fix = 0;
    size_t P = (size_t)g->T * o_plane(g);
    ALLOC_METRICS(g, P);
    if (kind == 0) {
        periodic_metrics(g);
    } else {
        if (connect(g, err, errlen)) { og_free(g); return NULL; }
        cube_metrics(g);
    }
    return g;
}

void og_free(OGrid *g)
{
    if (!g) return;
    double *m[] = {g->dx, g->dy, g->dxc, g->dyc, g->dxa, g->dya, g->area, g->area_c, g->fC,
                   g->fB, g->sin_u, g->cos_u, g->sin_v, g->cos_v, g->sin_a, g->cos_a,
                   g->cpos[0], g->cpos[1], g->cpos[2], g->bpos[0], g->bpos[1], g->bpos[2]};
    for (size_t q = 0; q < sizeof(m) / sizeof(m[0]); q++) free(m[q]);
    free(g);
}
