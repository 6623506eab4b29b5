// Coarse-grid support of the learned per-column correction: conservative
// coarsening of a cubed-sphere state by an integer factor, normalised column
// features for the network, and the application of predicted tendencies to a
// coarse state with a device-side fallback flag.
//
// All three are one-pass element kernels bound by HBM traffic; none is on the
// acoustic-substep path.
#include <cmath>
#include <string>

#include "fv3_internal.hpp"

namespace fv3 {
namespace {

__device__ __forceinline__ long at(const Geo &G, int L, int t, int k, int j, int i)
{
    return G.off0 + ((long)t * L + k) * G.lev + (long)j * G.pitch + i;
}

// cell fields over r x r blocks: delp and delz area means, pt and w
// mass-weighted means; FP64 sums
template <class B>
__global__ void k_coarsen_cells(Geo F, Geo C, int r, const double *__restrict__ areaf,
                                const double *__restrict__ areac, const B *__restrict__ delp,
                                const B *__restrict__ pt, const B *__restrict__ w,
                                const double *__restrict__ delz, B *cdelp, B *cpt, B *cw, double *cdelz)
{
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I >= C.n || J >= C.n) return;
    int t = blockIdx.z / C.nz, k = blockIdx.z % C.nz;
    double m = 0.0, md = 0.0, mt = 0.0, mw = 0.0;
    for (int b = 0; b < r; b++)
        for (int a = 0; a < r; a++) {
            int j = r * J + b, i = r * I + a;
            double A = areaf[at(F, 1, t, 0, j, i)];
            long e = at(F, F.nz, t, k, j, i);
            double mass = (double)delp[e] * A;
            m += mass;
            md += delz[e] * A;
            mt += (double)pt[e] * mass;
            mw += (double)w[e] * mass;
        }
    double Ac = areac[at(C, 1, t, 0, J, I)];
    long ce = at(C, C.nz, t, k, J, I);
    cdelp[ce] = (B)(m / Ac);
    cdelz[ce] = md / Ac;
    cpt[ce] = (B)(mt / m);
    cw[ce] = (B)(mw / m);
}

// D-grid winds: each coarse edge takes the edge-length-weighted mean of the
// r fine edges it is made of (the circulation along it is kept)
template <class B>
__global__ void k_coarsen_winds(Geo F, Geo C, int r, const double *__restrict__ dxf,
                                const double *__restrict__ dyf, const B *__restrict__ u,
                                const B *__restrict__ v, B *cu, B *cv)
{
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > C.n || J > C.n) return;
    int t = blockIdx.z / C.nz, k = blockIdx.z % C.nz;
    if (I < C.n) {   // y-face (I, J)
        double num = 0.0, den = 0.0;
        for (int a = 0; a < r; a++) {
            int j = r * J, i = r * I + a;
            double l = dxf[at(F, 1, t, 0, j, i)];
            num += (double)u[at(F, F.nz, t, k, j, i)] * l;
            den += l;
        }
        cu[at(C, C.nz, t, k, J, I)] = (B)(num / den);
    }
    if (J < C.n) {   // x-face (I, J)
        double num = 0.0, den = 0.0;
        for (int b = 0; b < r; b++) {
            int j = r * J + b, i = r * I;
            double l = dyf[at(F, 1, t, 0, j, i)];
            num += (double)v[at(F, F.nz, t, k, j, i)] * l;
            den += l;
        }
        cv[at(C, C.nz, t, k, J, I)] = (B)(num / den);
    }
}

// X[row][c] = (x - mean[c]) * inv_std[c]; rows ordered (tile, j, i), columns
// (field, level) with fields ua, va, pt, w, delp.  A value outside
// [lo - 6, hi + 6] (normalised units) or not finite sets bit 0 of *flag.
template <class B>
__global__ void k_features(Geo G, const B *__restrict__ u, const B *__restrict__ v, const B *__restrict__ pt,
                           const B *__restrict__ w, const B *__restrict__ delp, const float *__restrict__ mean,
                           const float *__restrict__ inv_std, const float *__restrict__ lo,
                           const float *__restrict__ hi, float *X, int *flag)
{
    const int n = G.n, nz = G.nz, F = 5 * nz;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = (long)G.T * n * n * F;
    if (e >= total) return;
    long row = e / F;
    int c = (int)(e % F);
    int f = c / nz, k = c % nz;
    int i = (int)(row % n), j = (int)((row / n) % n), t = (int)(row / ((long)n * n));
    double x;
    switch (f) {
    case 0: x = 0.5 * ((double)u[at(G, nz, t, k, j, i)] + (double)u[at(G, nz, t, k, j + 1, i)]); break;
    case 1: x = 0.5 * ((double)v[at(G, nz, t, k, j, i)] + (double)v[at(G, nz, t, k, j, i + 1)]); break;
    case 2: x = (double)pt[at(G, nz, t, k, j, i)]; break;
    case 3: x = (double)w[at(G, nz, t, k, j, i)]; break;
    default: x = (double)delp[at(G, nz, t, k, j, i)]; break;
    }
    float z = (float)((x - (double)mean[c]) * (double)inv_std[c]);
    X[e] = z;
    if (flag && !(z >= lo[c] - 6.0f && z <= hi[c] + 6.0f)) atomicOr(flag, 1);
}

__global__ void k_corr_check(const float *__restrict__ Y, long count, int *flag)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    if (!isfinite(Y[e])) atomicOr(flag, 2);
}

// physical tendencies from normalised outputs; pt updated in place, the wind
// increments (tile components, at cells) stored for the face pass
template <class B>
__global__ void k_corr_cells(Geo G, const float *__restrict__ Y, const float *__restrict__ ymean,
                             const float *__restrict__ ystd, double seconds, const int *__restrict__ flag,
                             B *pt, double *dU, double *dV)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= G.n || j >= G.n) return;
    if (*flag) return;
    int t = blockIdx.z / G.nz, k = blockIdx.z % G.nz, nz = G.nz;
    long row = ((long)t * G.n + j) * G.n + i;
    const float *y = Y + row * 3 * nz;
    double du = (double)y[k] * ystd[k] + ymean[k];
    double dv = (double)y[nz + k] * ystd[nz + k] + ymean[nz + k];
    double dp = (double)y[2 * nz + k] * ystd[2 * nz + k] + ymean[2 * nz + k];
    long e = at(G, nz, t, k, j, i);
    dU[e] = seconds * du;
    dV[e] = seconds * dv;
    pt[e] = (B)((double)pt[e] + seconds * dp);
}

// D-grid u on y-faces and v on x-faces take the mean increment of the two
// cells that share the face (the neighbour tile's cell through the halo)
template <class B>
__global__ void k_corr_faces(Geo G, const int *__restrict__ flag, const double *__restrict__ dU,
                             const double *__restrict__ dV, B *u, B *v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > G.n || j > G.n) return;
    if (*flag) return;
    int t = blockIdx.z / G.nz, k = blockIdx.z % G.nz, nz = G.nz;
    if (i < G.n) {
        long e = at(G, nz, t, k, j, i);
        u[e] = (B)((double)u[e] + 0.5 * (dU[at(G, nz, t, k, j - 1, i)] + dU[e]));
    }
    if (j < G.n) {
        long e = at(G, nz, t, k, j, i);
        v[e] = (B)((double)v[e] + 0.5 * (dV[at(G, nz, t, k, j, i - 1)] + dV[e]));
    }
}

template <class B>
void coarsen_t(const fv3_state *f, const fv3_grid *gf, fv3_state *c, const fv3_grid *gc, hipStream_t st)
{
    int r = gf->n / gc->n;
    dim3 blk(64, 4), grd((unsigned)((gc->n + 64) / 64), (unsigned)((gc->n + 4) / 4), (unsigned)(gc->T * gc->nz));
    hipLaunchKernelGGL(k_coarsen_cells<B>, grd, blk, 0, st, gf->geo, gc->geo, r, (const double *)gf->met[M_AREA],
                       (const double *)gc->met[M_AREA], (const B *)f->delp, (const B *)f->pt, (const B *)f->w,
                       (const double *)f->delz, (B *)c->delp, (B *)c->pt, (B *)c->w, c->delz);
    hipLaunchKernelGGL(k_coarsen_winds<B>, grd, blk, 0, st, gf->geo, gc->geo, r, (const double *)gf->met[M_DX],
                       (const double *)gf->met[M_DY], (const B *)f->u, (const B *)f->v, (B *)c->u, (B *)c->v);
}

template <class B>
void features_t(const fv3_state *s, const fv3_grid *g, const fv3_feature_norm *nm, float *X, int *flag,
                hipStream_t st)
{
    long total = (long)g->T * g->n * g->n * 5 * g->nz;
    hipLaunchKernelGGL(k_features<B>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g->geo,
                       (const B *)s->u, (const B *)s->v, (const B *)s->pt, (const B *)s->w, (const B *)s->delp,
                       nm->mean, nm->inv_std, nm->lo, nm->hi, X, flag);
}

template <class B>
fv3_status correct_t(fv3_state *s, const fv3_grid *g, const float *Y, const float *ymean, const float *ystd,
                     double seconds, int *flag, hipStream_t st)
{
    long el = alloc_elems(g, g->nz);
    double *dU = (double *)s->workspace, *dV = dU + el;
    long rows = (long)g->T * g->n * g->n, count = rows * 3 * g->nz;
    hipLaunchKernelGGL(k_corr_check, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, Y, count, flag);
    dim3 blk(64, 4);
    dim3 gc((unsigned)((g->n + 63) / 64), (unsigned)((g->n + 3) / 4), (unsigned)(g->T * g->nz));
    hipLaunchKernelGGL(k_corr_cells<B>, gc, blk, 0, st, g->geo, Y, ymean, ystd, seconds, (const int *)flag,
                       (B *)s->pt, dU, dV);
    fv3_status r = run_halo_pair_cells(g, dU, dV, g->nz, 1, st);
    if (r != FV3_OK) return r;
    dim3 gf((unsigned)((g->n + 64) / 64), (unsigned)((g->n + 4) / 4), (unsigned)(g->T * g->nz));
    hipLaunchKernelGGL(k_corr_faces<B>, gf, blk, 0, st, g->geo, (const int *)flag, (const double *)dU,
                       (const double *)dV, (B *)s->u, (B *)s->v);
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

}  // namespace
}  // namespace fv3

using namespace fv3;

extern "C" {

fv3_status fv3_coarsen(const fv3_state *fine, const fv3_grid *gf, fv3_state *coarse, const fv3_grid *gc,
                       void *stream)
{
    if (!fine || !gf || !coarse || !gc) return set_error(FV3_EINVAL, "NULL argument");
    const void *req[] = {fine->u, fine->v, fine->w, fine->delp, fine->pt, fine->delz,
                         coarse->u, coarse->v, coarse->w, coarse->delp, coarse->pt, coarse->delz};
    for (const void *p : req)
        if (!p) return set_error(FV3_EINVAL, "NULL field");
    if (gf->T != gc->T || gf->nz != gc->nz || gc->n < 1 || gf->n % gc->n != 0 || gf->n < gc->n)
        return set_error(FV3_ESHAPE, "fine grid must have the coarse grid's tiles and levels and n = r * n_coarse");
    if (gf->p.kind != gc->p.kind) return set_error(FV3_ESHAPE, "grid kinds differ");
    if (gf->bulk_bytes != gc->bulk_bytes) return set_error(FV3_EDTYPE, "grids of different precision");
    if (!device_current(gf) || !device_current(gc))
        return set_error(FV3_EDEVICE, "current HIP device differs from the grid's device");
    hipStream_t st = (hipStream_t)stream;
    if (gf->bulk_bytes == 4) coarsen_t<float>(fine, gf, coarse, gc, st);
    else coarsen_t<double>(fine, gf, coarse, gc, st);
    return hipGetLastError() == hipSuccess ? FV3_OK : set_error(FV3_EDEVICE, "launch failed");
}

fv3_status fv3_column_features(const fv3_state *s, const fv3_grid *g, const fv3_feature_norm *norm, float *X,
                               int *flag, void *stream)
{
    if (!s || !g || !norm || !X) return set_error(FV3_EINVAL, "NULL argument");
    if (!s->u || !s->v || !s->pt || !s->w || !s->delp) return set_error(FV3_EINVAL, "NULL field");
    if (!norm->mean || !norm->inv_std || (flag && (!norm->lo || !norm->hi)))
        return set_error(FV3_EINVAL, "NULL normalisation array");
    if (!device_current(g)) return set_error(FV3_EDEVICE, "current HIP device differs from the grid's device");
    hipStream_t st = (hipStream_t)stream;
    if (g->bulk_bytes == 4) features_t<float>(s, g, norm, X, flag, st);
    else features_t<double>(s, g, norm, X, flag, st);
    return hipGetLastError() == hipSuccess ? FV3_OK : set_error(FV3_EDEVICE, "launch failed");
}

fv3_status fv3_apply_correction(fv3_state *s, const fv3_grid *g, const float *Y, const float *ymean,
                                const float *ystd, double seconds, int *flag, void *stream)
{
    if (!s || !g || !Y || !ymean || !ystd || !flag) return set_error(FV3_EINVAL, "NULL argument");
    if (!s->u || !s->v || !s->pt || !s->workspace) return set_error(FV3_EINVAL, "NULL field or workspace");
    if (!std::isfinite(seconds)) return set_error(FV3_EINVAL, "seconds must be finite");
    size_t need = 2 * (size_t)alloc_elems(g, g->nz) * sizeof(double);
    if (s->workspace_bytes < need) return set_error(FV3_EINVAL, "workspace too small");
    if (!device_current(g)) return set_error(FV3_EDEVICE, "current HIP device differs from the grid's device");
    hipStream_t st = (hipStream_t)stream;
    fv3_status r = g->bulk_bytes == 4 ? correct_t<float>(s, g, Y, ymean, ystd, seconds, flag, st)
                                      : correct_t<double>(s, g, Y, ymean, ystd, seconds, flag, st);
    return r == FV3_OK ? FV3_OK : set_error(r, "launch failed");
}

}  // extern "C"
