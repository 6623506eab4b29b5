/*
 * FV3 acoustic-substep ORACLE -- test infrastructure only.
 *
 * A plain, slow, FP64 CPU implementation of the nonhydrostatic acoustic
 * substep loop and tracer transport of the FV3 dynamical core (the innermost
 * and middle loops of the three-level substepping, paper Sec. II), written to
 * be checked by eye against the method.  Only the test suite, the smoke entry
 * point and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library; the two are compared
 * element by element on the same seeded inputs.
 *
 * Layout used throughout the oracle (deliberately unpadded and simple):
 *   3-D field  f[t][k][jj][ii],  jj = j + H, ii = i + H,  N = n + 2H + 1
 *   2-D metric m[t][jj][ii]
 * with H = 3 halo points on every side.  Staggerings share the N x N plane:
 *   C  cell centre   (i+1/2, j+1/2)     interior i,j in [0,n-1]
 *   X  x-face        (i,     j+1/2)     interior i in [0,n], j in [0,n-1]
 *   Y  y-face        (i+1/2, j    )     interior i in [0,n-1], j in [0,n]
 *   B  cell corner   (i,     j    )     interior i,j in [0,n]
 * (coordinates in units of the grid spacing, corner (0,0) at the tile's SW
 * vertex).  D-grid winds: u on Y, v on X.  C-grid winds: uc on X, vc on Y.
 */
#ifndef FV3_ORACLE_ORC_H
#define FV3_ORACLE_ORC_H

#include <stddef.h>

#define H 3

enum { ST_C = 0, ST_X = 1, ST_Y = 2, ST_B = 3 };
enum { MODE_X = 0, MODE_Y = 1 };
/* how a pair of components transforms when copied across a rotated edge */
enum { PAIR_SIGNED = 0, PAIR_ABS = 1, PAIR_COS = 2 };

/* physical constants of the dry nonhydrostatic system (reading R3) */
#define O_GRAV 9.80665
#define O_RDGAS 287.05
#define O_CP 1004.6
#define O_P0 1.0e5
#define O_RVGAS 461.5

typedef struct {
    int kind;              /* 0 doubly periodic, 1 cubed sphere */
    int n, nz, T, N;
    double delta, f0, radius, omega, ptop;
    /* optional del-2 divergence damping of d_sw: coefficient and the smallest
     * corner (dual-cell) area of the grid */
    double d2_bg, da_min;
    /* off-centring weight of the vertical solve (1 = backward Euler) */
    double beta;
    /* Smagorinsky coefficient of the divergence damping (0 = off) */
    double dddmp;
    /* PPM order of every transport: 8 monotone (default), 6 unlimited,
     * 5 2dx-filtered; hord_tr that of the tracer transport (0: hord; also
     * 7, positive-definite) */
    int hord, hord_tr;
    /* interface perturbation of the column solves: 2 mass-linear (default), 4 cubic */
    int pp_order;
    /* higher-order divergence damping: order nord (1 del-4, 2 del-6, 0 off), coefficient d4_bg */
    int nord;
    double d4_bg;
    /* del-2 vorticity damping coefficient (0 = off) */
    double vtdm;
    /* cube: replace both tiles' fluxes through a shared edge face by their mean */
    int edge_fix;
    int edge_ppm;          /* one-sided PPM edge values at cube tile edges */
    int edge_interp;       /* one-sided c_sw and nh_p_grad interpolations at cube tile edges */
    /* cube connectivity: per tile, per edge (0 W, 1 E, 2 S, 3 N) */
    int nbr[6][4];
    int R[6][4][2][2];     /* lattice rotation from this tile into the neighbour */
    int P0[6][4][2];       /* edge start point on this tile (lattice units)      */
    int Q0[6][4][2];       /* the same point on the neighbour tile               */
    /* metrics [T][N][N]; halos hold the neighbour's values */
    double *dx, *dy, *dxc, *dyc, *dxa, *dya, *area, *area_c, *fC, *fB;
    double *sin_u, *cos_u, *sin_v, *cos_v, *sin_a, *cos_a;
    /* unit-sphere positions (cube only): cell centres and cell corners */
    double *cpos[3], *bpos[3];
} OGrid;

static inline size_t o_plane(const OGrid *g) { return (size_t)g->N * g->N; }

/* one-dimensional interpolations of c_sw and nh_p_grad (see dyn.c) */
enum { OI_FACE_PT = 0, OI_CELL_PT = 1, OI_FACE_MEAN = 2 };
double o_interp(int kind, const double *x0, ptrdiff_t s, int m0, int m, int n, int edge);
void o_corner_values(const OGrid *g, const double *q, double *qB);
double o_corner_vort(const OGrid *g, int t, const double *ucp, const double *vcp, int i, int j);
void o_corner_vort_all(const OGrid *g, const double *uc, const double *vc, double *out);
#define IX(g, i, j) ((size_t)((j) + H) * (size_t)(g)->N + (size_t)((i) + H))

/* caller-owned state arrays of the substep loop */
typedef struct {
    double *u, *v, *w, *delp, *pt, *delz, *uc, *vc, *mfx, *mfy, *cx, *cy, *dp0, *pfull, *phi;
    const double *phis;
    double *qv;   /* specific humidity (cell field) or NULL: dry */
} OState;

/* grid.c */
OGrid *og_new(int kind, int n, int nz, double delta, double f0, double radius,
              double omega, double ptop, char *err, size_t errlen);
void og_free(OGrid *g);

/* halo.c */
int og_region(const OGrid *g, int st, int i, int j);   /* 0 interior, 1 edge halo, 2 corner block */
void og_fill_scalar(const OGrid *g, double *f, int nlev, int st, int coslike);
void og_fill_pair(const OGrid *g, double *fx, int stx, double *fy, int sty, int nlev, int kind);
void og_view_scalar(const OGrid *g, const double *plane, int st, int mode, int coslike, double *out);
void og_view_pair(const OGrid *g, const double *px, int stx, const double *py, int sty,
                  int mode, int kind, double *ox, double *oy);
int og_is_vertex(const OGrid *g, int i, int j);
int og_edge_partner(const OGrid *g, int t, int st, int i, int j, int *tp, int *stp, int *ip, int *jp);

/* ppm.c */
double o_ppm_face(const double q[6], double c);
double o_ppm_face_edge(const double q[6], const double w[6], double c, int ord, int pe, int west);
double o_ppm_face_wind(const OGrid *g, const double q[6], const double w[6], double c, int ord, int m);
double o_ppm_face_order(const double q[6], double c, int ord);
void o_fv_tp_2d_ord(const OGrid *g, int ord, int t, const double *q, const double *qx, const double *qy,
                    const double *crx, const double *cry, const double *xfx, const double *yfx,
                    const double *mx, const double *my, double *FX, double *FY);
void o_fv_tp_2d(const OGrid *g, int t, const double *q, const double *qx, const double *qy,
                const double *crx, const double *cry, const double *xfx, const double *yfx,
                const double *mx, const double *my, double *FX, double *FY);

/* column.c */
double o_sim1(int nz, double dt, double ptop, double zs, const double *dpi, const double *theta,
              const double *delz, const double *w, double *w_out, double *delz_out,
              double *pfull, double *phi);
/* off-centred form (beta in [0.5, 1]); pstar / coupling (nz + 1, may be NULL)
 * receive the interface perturbation P* and the unscaled coupling dt x the
 * linearised pressure response */
double o_sim1b(int nz, double dt, double beta, int pp_order, double ptop, double zs, const double *dpi,
               const double *theta, const double *delz, const double *w, double *w_out,
               double *delz_out, double *pfull, double *phi, double *pstar, double *coupling);
void o_pp_interfaces(int nz, int order, const double *dpi, const double *pp, double *pps);
void o_corner_div(const OGrid *g, int t, const double *U, const double *V, double *out);
void o_corner_lap(const OGrid *g, int t, const double *D, double *out);
void o_edge_fix_dsw(const OGrid *g, const double *FXm, const double *FYm, const double *FXp,
                    const double *FYp, const double *FXw, const double *FYw, double *delp, double *pt,
                    double *w, double *mfx, double *mfy);
void o_edge_fix_tracer(const OGrid *g, const double *FX, const double *FY, const double *dp2, double *q);
double o_pgf(double dt, double L, double dpiW, double dpiE, double phW0, double phW1,
             double phE0, double phE1, double pW0, double pW1, double pE0, double pE1);

/* dyn.c: Smagorinsky magnitude dt sqrt(DT^2 + DS^2) at the corners of one level */
void o_smag_corner(const OGrid *g, int t, const double *u, const double *v, double dt, double *out);

/* remap.c */
void o_ppm_edges(int nz, const double *d, const double *a, double *e);
void o_ppm_profile(int nz, const double *d, const double *a, double *aL, double *aR, double *a6);
void o_remap_column(int nz, const double *pe1, const double *pe2, const double *q1, double *q2);
int orc_remap_impl(const OGrid *g, double *u, double *v, double *w, double *delp, double *pt,
                   double *delz, double *const *q, int nq, const double *ak, const double *bk);

#endif
