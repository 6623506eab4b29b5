/*
 * ORACLE (test infrastructure only): flat C entry points loaded by the
 * Python test helpers through ctypes.  Plain host pointers in the oracle's
 * own unpadded layout (see orc.h); nothing here is used by the library.
 */
#include "orc.h"
#include <stdlib.h>
#include <string.h>


int orc_substeps_impl(const OGrid *g, OState *s, double dt, int n_split, int stop_stage,
                      double **dbg);
int orc_tracer_impl(const OGrid *g, double **q, int nq, const double *dp0, const double *mfx,
                    const double *mfy, const double *cx, const double *cy, int nsplt,
                    int *nsplt_used);
void orc_mass_sums_impl(const OGrid *g, const double *delp, const double *pt,
                        const double *const *q, int nq, double *out);

void *orc_grid_new(int kind, int n, int nz, double delta, double f0, double radius,
                   double omega, double ptop, char *err, int errlen)
{
    return og_new(kind, n, nz, delta, f0, radius, omega, ptop, err, (size_t)errlen);
}

void orc_grid_free(void *g) { og_free((OGrid *)g); }

/* del-2 divergence damping of d_sw (0 = off) */
void orc_set_damping(void *gp, double d2_bg)
{
    OGrid *g = (OGrid *)gp;
    g->d2_bg = d2_bg;
    double m = 1e300;
    for (int t = 0; t < g->T; t++)
        for (int j = 0; j <= g->n; j++)
            for (int i = 0; i <= g->n; i++) {
                double a = g->area_c[(size_t)t * o_plane(g) + IX(g, i, j)];
                if (a < m) m = a;
            }
    g->da_min = m;
}

/* Smagorinsky coefficient of the divergence damping */
void orc_set_smag(void *gp, double dddmp) { ((OGrid *)gp)->dddmp = dddmp; }
void orc_set_vtdm(void *gp, double vtdm) { ((OGrid *)gp)->vtdm = vtdm; }
void orc_set_edge_fix(void *gp, int on) { ((OGrid *)gp)->edge_fix = on; }
void orc_set_edge_ppm(void *gp, int on) { ((OGrid *)gp)->edge_ppm = on; }
void orc_set_edge_interp(void *gp, int on) { ((OGrid *)gp)->edge_interp = on; }

void orc_corner_values(void *gp, const double *q, double *qB) { o_corner_values((const OGrid *)gp, q, qB); }
void orc_corner_vort(void *gp, const double *uc, const double *vc, double *out)
{
    o_corner_vort_all((const OGrid *)gp, uc, vc, out);
}

double orc_interp(int kind, const double *x, int len, int m0, int m, int n, int edge)
{
    (void)len;
    return o_interp(kind, x, 1, m0, m, n, edge);
}

int orc_edge_partner(void *gp, int t, int st, int i, int j, int *out4)
{
    return og_edge_partner((const OGrid *)gp, t, st, i, j, out4, out4 + 1, out4 + 2, out4 + 3);
}

void orc_set_damp4(void *gp, int nord, double d4_bg)
{
    ((OGrid *)gp)->nord = nord;
    ((OGrid *)gp)->d4_bg = d4_bg;
}

/* corner divergence / Laplacian of whole fields (all tiles, nlev planes);
 * the Laplacian fills the corner halo of its input first */
void orc_corner_div(void *gp, int nlev, const double *U, const double *V, double *out)
{
    const OGrid *g = (const OGrid *)gp;
    size_t P = o_plane(g);
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nlev; k++) {
            size_t q = ((size_t)t * nlev + k) * P;
            o_corner_div(g, t, U + q, V + q, out + q);
        }
}

void orc_corner_lap(void *gp, int nlev, double *D, double *out)
{
    const OGrid *g = (const OGrid *)gp;
    size_t P = o_plane(g);
    og_fill_scalar(g, D, nlev, ST_B, 0);
    for (int t = 0; t < g->T; t++)
        for (int k = 0; k < nlev; k++) {
            size_t q = ((size_t)t * nlev + k) * P;
            o_corner_lap(g, t, D + q, out + q);
        }
}

/* Smagorinsky magnitude of one level (oracle plane layout, halos filled) */
void orc_smag_corner(void *gp, int t, const double *u, const double *v, double dt, double *out)
{
    o_smag_corner((const OGrid *)gp, t, u, v, dt, out);
}

/* off-centring weight of the vertical solve */
void orc_set_beta(void *gp, double beta) { ((OGrid *)gp)->beta = beta; }

/* which: 0 dx 1 dy 2 dxc 3 dyc 4 dxa 5 dya 6 area 7 area_c 8 fC 9 fB 10 sin_u 11 cos_u
 *        12 sin_v 13 cos_v 14 sin_a 15 cos_a 16..18 centre xyz 19..21 corner xyz */
int orc_grid_metric(void *gp, int which, double *out)
{
    OGrid *g = (OGrid *)gp;
    double *m[] = {g->dx, g->dy, g->dxc, g->dyc, g->dxa, g->dya, g->area, g->area_c, g->fC,
                   g->fB, g->sin_u, g->cos_u, g->sin_v, g->cos_v, g->sin_a, g->cos_a,
                   g->cpos[0], g->cpos[1], g->cpos[2], g->bpos[0], g->bpos[1], g->bpos[2]};
    if (which < 0 || which >= (int)(sizeof(m) / sizeof(m[0])) || !m[which]) return -1;
    memcpy(out, m[which], sizeof(double) * g->T * o_plane(g));
    return 0;
}

int orc_grid_conn(void *gp, int *nbr, int *rot)
{
    OGrid *g = (OGrid *)gp;
    if (g->kind != 1) return -1;
    for (int t = 0; t < 6; t++)
        for (int e = 0; e < 4; e++) {
            nbr[t * 4 + e] = g->nbr[t][e];
            memcpy(rot + (t * 4 + e) * 4, g->R[t][e], sizeof(int) * 4);
        }
    return 0;
}

int orc_halo_fill(void *gp, double *f, int nlev, int st, int coslike)
{
    og_fill_scalar((OGrid *)gp, f, nlev, st, coslike);
    return 0;
}

int orc_halo_fill_pair(void *gp, double *fx, int stx, double *fy, int sty, int nlev, int kind)
{
    og_fill_pair((OGrid *)gp, fx, stx, fy, sty, nlev, kind);
    return 0;
}

int orc_corner_view(void *gp, const double *plane, int st, int mode, double *out)
{
    og_view_scalar((OGrid *)gp, plane, st, mode, 0, out);
    return 0;
}

int orc_corner_view_pair(void *gp, const double *px, int stx, const double *py, int sty,
                         int mode, double *ox, double *oy)
{
    og_view_pair((OGrid *)gp, px, stx, py, sty, mode, PAIR_SIGNED, ox, oy);
    return 0;
}

double orc_ppm_face(const double *q6, double c) { return o_ppm_face(q6, c); }
double orc_ppm_face_order(const double *q6, double c, int ord) { return o_ppm_face_order(q6, c, ord); }
double orc_ppm_face_edge(const double *q6, const double *w6, double c, int ord, int pe, int west)
{
    return o_ppm_face_edge(q6, w6, c, ord, pe, west);
}
void orc_set_hord(void *gp, int hord, int hord_tr)
{
    ((OGrid *)gp)->hord = hord;
    ((OGrid *)gp)->hord_tr = hord_tr;
}

int orc_fv_tp_2d(void *gp, int t, const double *q, const double *crx, const double *cry,
                 const double *xfx, const double *yfx, const double *mx, const double *my,
                 double *FX, double *FY)
{
    OGrid *g = (OGrid *)gp;
    size_t P = o_plane(g);
    double *qx = (double *)malloc(P * sizeof(double)), *qy = (double *)malloc(P * sizeof(double));
    og_view_scalar(g, q, ST_C, MODE_X, 0, qx);
    og_view_scalar(g, q, ST_C, MODE_Y, 0, qy);
    o_fv_tp_2d(g, t, q, qx, qy, crx, cry, xfx, yfx, mx, my, FX, FY);
    free(qx); free(qy);
    return 0;
}

double orc_sim1(int nz, double dt, double ptop, double zs, const double *dpi, const double *theta,
                const double *delz, const double *w, double *w_out, double *delz_out,
                double *pfull, double *phi)
{
    return o_sim1(nz, dt, ptop, zs, dpi, theta, delz, w, w_out, delz_out, pfull, phi);
}

double orc_sim1b(int nz, double dt, double beta, int pp_order, double ptop, double zs, const double *dpi,
                 const double *theta, const double *delz, const double *w, double *w_out,
                 double *delz_out, double *pfull, double *phi, double *pstar, double *coupling)
{
    return o_sim1b(nz, dt, beta, pp_order, ptop, zs, dpi, theta, delz, w, w_out, delz_out, pfull, phi, pstar,
                   coupling);
}

void orc_pp_interfaces(int nz, int order, const double *dpi, const double *pp, double *pps)
{
    o_pp_interfaces(nz, order, dpi, pp, pps);
}

void orc_set_pp_order(void *gp, int order) { ((OGrid *)gp)->pp_order = order; }

double orc_pgf(double dt, double L, double dpiW, double dpiE, double phW0, double phW1,
               double phE0, double phE1, double pW0, double pW1, double pE0, double pE1)
{
    return o_pgf(dt, L, dpiW, dpiE, phW0, phW1, phE0, phE1, pW0, pW1, pE0, pE1);
}

int orc_acoustic_substeps(void *gp, double *u, double *v, double *w, double *delp, double *pt,
                          double *delz, double *uc, double *vc, double *mfx, double *mfy,
                          double *cx, double *cy, double *dp0, double *pfull, double *phi,
                          const double *phis, double *qv, double dt, int n_split, int stop_stage,
                          double **dbg)
{
    OState s = {u, v, w, delp, pt, delz, uc, vc, mfx, mfy, cx, cy, dp0, pfull, phi, phis, qv};
    if (n_split < 1 || !(dt > 0)) return -1;
    return orc_substeps_impl((OGrid *)gp, &s, dt, n_split, stop_stage, dbg);
}

int orc_tracer_transport(void *gp, double **q, int nq, const double *dp0, const double *mfx,
                         const double *mfy, const double *cx, const double *cy, int nsplt,
                         int *nsplt_used)
{
    return orc_tracer_impl((OGrid *)gp, q, nq, dp0, mfx, mfy, cx, cy, nsplt, nsplt_used);
}

int orc_mass_sums(void *gp, const double *delp, const double *pt, const double *const *q, int nq,
                  double *out)
{
    orc_mass_sums_impl((OGrid *)gp, delp, pt, q, nq, out);
    return 0;
}

void orc_ppm_edges(int nz, const double *d, const double *a, double *e) { o_ppm_edges(nz, d, a, e); }

void orc_ppm_profile(int nz, const double *d, const double *a, double *aL, double *aR, double *a6)
{
    o_ppm_profile(nz, d, a, aL, aR, a6);
}

void orc_remap_column(int nz, const double *pe1, const double *pe2, const double *q1, double *q2)
{
    o_remap_column(nz, pe1, pe2, q1, q2);
}

int orc_remap(void *gp, double *u, double *v, double *w, double *delp, double *pt, double *delz,
              double *const *q, int nq, const double *ak, const double *bk)
{
    return orc_remap_impl((OGrid *)gp, u, v, w, delp, pt, delz, q, nq, ak, bk);
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
    return n;
#else
    (void)n;
    return 1;
#endif
}
