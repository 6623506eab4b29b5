/*
 * ORACLE (test infrastructure only): halo fills and cube-corner views.
 *
 * Halo exchange between subdomains with the orientation transform between
 * adjoining cube faces follows the paper's halo-updater description
 * (Sec. V-C); here all six tiles live in one address space so a "halo
 * exchange" is a copy from the neighbour tile's interior.  The 3x3 corner
 * blocks at cube vertices have no owner (only three faces meet there); they
 * are never stored.  A consumer reads them through a "view" that rotates the
 * adjacent edge halo about the vertex, in the x-sweep or y-sweep sense, which
 * generalises the corner statement printed in Sec. VII-C (the SW cell
 * (-1,-1) takes the value of cell (-1,0)).
 *
 * Geometry is handled in doubled lattice coordinates: a point of stagger st
 * at storage index (i,j) sits at (2i+sx, 2j+sy) with (sx,sy) = (1,1) for C,
 * (0,1) for X, (1,0) for Y, (0,0) for B.
 */
#include "orc.h"
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static const int SX[4] = {1, 0, 1, 0};
static const int SY[4] = {1, 1, 0, 0};

static int floordiv2(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

static int stag_of(int x2, int y2)
{
    int ox = x2 & 1, oy = y2 & 1;
    if (ox && oy) return ST_C;
    if (!ox && oy) return ST_X;
    if (ox && !oy) return ST_Y;
    return ST_B;
}

static void st_range(const OGrid *g, int st, int *ilo, int *ihi, int *jlo, int *jhi)
{
    int n = g->n;
    *ilo = -H; *jlo = -H;
    *ihi = (st == ST_X || st == ST_B) ? n + H : n + H - 1;
    *jhi = (st == ST_Y || st == ST_B) ? n + H : n + H - 1;
}

int og_region(const OGrid *g, int st, int i, int j)
{
    int x2 = 2 * i + SX[st], y2 = 2 * j + SY[st], n2 = 2 * g->n;
    int inx = (x2 >= 0 && x2 <= n2), iny = (y2 >= 0 && y2 <= n2);
    if (inx && iny) return 0;
    if (inx || iny) return 1;
    return 2;
}

int og_is_vertex(const OGrid *g, int i, int j)
{
    return g->kind == 1 && (i == 0 || i == g->n) && (j == 0 || j == g->n);
}

/* Source of an edge-halo point (or, on the periodic grid, any halo point):
 * tile, doubled coordinates and the lattice rotation applied to vectors. */
static void halo_source(const OGrid *g, int t, int x2, int y2, int *ts, int *qx2, int *qy2,
                        int R[2][2])
{
    int n2 = 2 * g->n;
    if (g->kind == 0) {
        *ts = t;
        *qx2 = x2 < 0 ? x2 + n2 : (x2 > n2 ? x2 - n2 : x2);
        *qy2 = y2 < 0 ? y2 + n2 : (y2 > n2 ? y2 - n2 : y2);
        R[0][0] = 1; R[0][1] = 0; R[1][0] = 0; R[1][1] = 1;
        return;
    }
    int e;
    if (x2 < 0) e = 0;
    else if (x2 > n2) e = 1;
    else if (y2 < 0) e = 2;
    else e = 3;
    *ts = g->nbr[t][e];
    memcpy(R, g->R[t][e], sizeof(int) * 4);
    int dx = x2 - 2 * g->P0[t][e][0], dy = y2 - 2 * g->P0[t][e][1];
    *qx2 = R[0][0] * dx + R[0][1] * dy + 2 * g->Q0[t][e][0];
    *qy2 = R[1][0] * dx + R[1][1] * dy + 2 * g->Q0[t][e][1];
}

static void must_interior(const OGrid *g, int x2, int y2)
{
    int n2 = 2 * g->n;
    if (x2 < 0 || x2 > n2 || y2 < 0 || y2 > n2) {
        fprintf(stderr, "oracle halo: source (%d,%d) outside the interior\n", x2, y2);
        abort();
    }
}

/* Which source component (0 = x, 1 = y) and sign a unit direction maps to. */
static void rot_dir(int R[2][2], int dir, int *comp, int *sign)
{
    int vx = dir == 0 ? R[0][0] : R[0][1];
    int vy = dir == 0 ? R[1][0] : R[1][1];
    if (vx != 0) { *comp = 0; *sign = vx; }
    else { *comp = 1; *sign = vy; }
}

static int cos_sign(int R[2][2])
{
    int c0, s0, c1, s1;
    rot_dir(R, 0, &c0, &s0);
    rot_dir(R, 1, &c1, &s1);
    return s0 * s1;
}

void og_fill_scalar(const OGrid *g, double *f, int nlev, int st, int coslike)
{
    size_t P = o_plane(g);
    int ilo, ihi, jlo, jhi;
    st_range(g, st, &ilo, &ihi, &jlo, &jhi);
    for (int t = 0; t < g->T; t++)
        for (int j = jlo; j <= jhi; j++)
            for (int i = ilo; i <= ihi; i++) {
                int reg = og_region(g, st, i, j);
                if (reg == 0) continue;
                if (reg == 2 && g->kind == 1) continue;   /* cube corner blocks: views only */
                int ts, qx2, qy2, R[2][2];
                halo_source(g, t, 2 * i + SX[st], 2 * j + SY[st], &ts, &qx2, &qy2, R);
                must_interior(g, qx2, qy2);
                int qi = floordiv2(qx2), qj = floordiv2(qy2);
                double s = coslike ? (double)cos_sign(R) : 1.0;
                for (int k = 0; k < nlev; k++)
                    f[((size_t)t * nlev + k) * P + IX(g, i, j)] =
                        s * f[((size_t)ts * nlev + k) * P + IX(g, qi, qj)];
            }
}

static double pair_sign(int kind, int sign, int R[2][2])
{
    if (kind == PAIR_SIGNED) return (double)sign;
    if (kind == PAIR_ABS) return 1.0;
    return (double)cos_sign(R);
}

void og_fill_pair(const OGrid *g, double *fx, int stx, double *fy, int sty, int nlev, int kind)
{
    size_t P = o_plane(g);
    for (int comp = 0; comp < 2; comp++) {
        int st = comp == 0 ? stx : sty;
        double *dst = comp == 0 ? fx : fy;
        int ilo, ihi, jlo, jhi;
        st_range(g, st, &ilo, &ihi, &jlo, &jhi);
        for (int t = 0; t < g->T; t++)
            for (int j = jlo; j <= jhi; j++)
                for (int i = ilo; i <= ihi; i++) {
                    int reg = og_region(g, st, i, j);
                    if (reg == 0) continue;
                    if (reg == 2 && g->kind == 1) continue;
                    int ts, qx2, qy2, R[2][2];
                    halo_source(g, t, 2 * i + SX[st], 2 * j + SY[st], &ts, &qx2, &qy2, R);
                    must_interior(g, qx2, qy2);
                    int sc, sg;
                    rot_dir(R, comp, &sc, &sg);
                    int want = sc == 0 ? stx : sty;
                    if (stag_of(qx2, qy2) != want) {
                        fprintf(stderr, "oracle halo: stagger mismatch\n");
                        abort();
                    }
                    const double *src = sc == 0 ? fx : fy;
                    double s = pair_sign(kind, sg, R);
                    int qi = floordiv2(qx2), qj = floordiv2(qy2);
                    for (int k = 0; k < nlev; k++)
                        dst[((size_t)t * nlev + k) * P + IX(g, i, j)] =
                            s * src[((size_t)ts * nlev + k) * P + IX(g, qi, qj)];
                }
    }
}

/* Corner-view rotations about the cube vertex.  CW maps (x,y) -> (y,-x),
 * CCW maps (x,y) -> (-y,x).  Index: [mode][corner], corner 0 SW 1 SE 2 NW 3 NE.
 * x-sweep views borrow the W/E edge halo, y-sweep views the S/N one. */
static const int RCW[2][2] = {{0, 1}, {-1, 0}};
static const int RCCW[2][2] = {{0, -1}, {1, 0}};

static void corner_rot(int mode, int corner, int R[2][2])
{
    int cw;
    if (mode == MODE_X) cw = (corner == 0 || corner == 3);
    else cw = (corner == 1 || corner == 2);
    memcpy(R, cw ? RCW : RCCW, sizeof(int) * 4);
}

/* For a corner-block point of stagger st, find the edge-halo point it views. */
static void corner_source(const OGrid *g, int st, int i, int j, int mode, int *qi, int *qj,
                          int *qst, int R[2][2])
{
    int n2 = 2 * g->n;
    int x2 = 2 * i + SX[st], y2 = 2 * j + SY[st];
    int vx = x2 < 0 ? 0 : n2, vy = y2 < 0 ? 0 : n2;
    int corner = (x2 < 0 ? 0 : 1) + (y2 < 0 ? 0 : 2);
    corner_rot(mode, corner, R);
    int dx = x2 - vx, dy = y2 - vy;
    int qx2 = vx + R[0][0] * dx + R[0][1] * dy;
    int qy2 = vy + R[1][0] * dx + R[1][1] * dy;
    *qi = floordiv2(qx2);
    *qj = floordiv2(qy2);
    *qst = stag_of(qx2, qy2);
}

void og_view_scalar(const OGrid *g, const double *plane, int st, int mode, int coslike,
                    double *out)
{
    memcpy(out, plane, sizeof(double) * o_plane(g));
    if (g->kind == 0) return;
    int ilo, ihi, jlo, jhi;
    st_range(g, st, &ilo, &ihi, &jlo, &jhi);
    for (int j = jlo; j <= jhi; j++)
        for (int i = ilo; i <= ihi; i++) {
            if (og_region(g, st, i, j) != 2) continue;
            int qi, qj, qst, R[2][2];
            corner_source(g, st, i, j, mode, &qi, &qj, &qst, R);
            if (og_region(g, qst, qi, qj) != 1) abort();
            out[IX(g, i, j)] = (coslike ? cos_sign(R) : 1) * plane[IX(g, qi, qj)];
        }
}

void og_view_pair(const OGrid *g, const double *px, int stx, const double *py, int sty,
                  int mode, int kind, double *ox, double *oy)
{
    size_t P = o_plane(g);
    memcpy(ox, px, sizeof(double) * P);
    memcpy(oy, py, sizeof(double) * P);
    if (g->kind == 0) return;
    for (int comp = 0; comp < 2; comp++) {
        int st = comp == 0 ? stx : sty;
        double *dst = comp == 0 ? ox : oy;
        int ilo, ihi, jlo, jhi;
        st_range(g, st, &ilo, &ihi, &jlo, &jhi);
        for (int j = jlo; j <= jhi; j++)
            for (int i = ilo; i <= ihi; i++) {
                if (og_region(g, st, i, j) != 2) continue;
                int qi, qj, qst, R[2][2];
                corner_source(g, st, i, j, mode, &qi, &qj, &qst, R);
                int sc, sg;
                rot_dir(R, comp, &sc, &sg);
                if (qst != (sc == 0 ? stx : sty) || og_region(g, qst, qi, qj) != 1) abort();
                const double *src = sc == 0 ? px : py;
                dst[IX(g, i, j)] = pair_sign(kind, sg, R) * src[IX(g, qi, qj)];
            }
    }
}

/* The other tile's copy of a face on a tile edge of the cube: x-face (st =
 * ST_X, i = 0 or n) or y-face (ST_Y, j = 0 or n).  Writes the partner tile,
 * stagger and indices; returns the sign with which the partner's flux
 * (positive along its own +x or +y) counts along our +x or +y. */
int og_edge_partner(const OGrid *g, int t, int st, int i, int j, int *tp, int *stp, int *ip, int *jp)
{
    int n2 = 2 * g->n, x2 = 2 * i + SX[st], y2 = 2 * j + SY[st];
    int e;
    if (st == ST_X) e = x2 == 0 ? 0 : 1;
    else e = y2 == 0 ? 2 : 3;
    (void)n2;
    int R[2][2];
    memcpy(R, g->R[t][e], sizeof(int) * 4);
    int dx = x2 - 2 * g->P0[t][e][0], dy = y2 - 2 * g->P0[t][e][1];
    int qx2 = R[0][0] * dx + R[0][1] * dy + 2 * g->Q0[t][e][0];
    int qy2 = R[1][0] * dx + R[1][1] * dy + 2 * g->Q0[t][e][1];
    *tp = g->nbr[t][e];
    *stp = stag_of(qx2, qy2);
    *ip = floordiv2(qx2);
    *jp = floordiv2(qy2);
    int comp, sign;
    rot_dir(R, st == ST_X ? 0 : 1, &comp, &sign);
    return sign;
}
