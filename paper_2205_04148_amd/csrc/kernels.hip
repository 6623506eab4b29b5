// HIP kernels of the FV3 acoustic substep loop and tracer transport (gfx950).
//
// Data layout: every field is [tile][level][row][column], column index i
// contiguous (coalesced across the 64 lanes of a wavefront), halo of 3 points,
// rows padded to a multiple of 128 bytes with interior i = 0 aligned.  One
// kernel per stage of the method, each thread one output point of one
// (tile, level) plane; column solves march k in one thread per column with
// the column's unknowns in FP64.  Corner blocks of cube tiles are never
// stored: reads of them are remapped to the adjacent edge halo rotated about
// the cube vertex, in the x-sweep or y-sweep sense of the reading stencil
// (generalising the corner statement of Sec. VII-C).
//
// Stage formulas: see the method description in each kernel's comment; the
// order of the stages inside a substep follows the FV3 acoustic loop
// (Sec. II): halo A, c_sw, dz_c + riem_solver_c, p_grad_c, halo B, d_sw,
// dz_d + riem_solver3, halo C, nh_p_grad.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fv3_internal.hpp"

namespace fv3 {

typedef double B;   // bulk precision of this build of the kernels

#define DEVI __device__ __forceinline__

// ------------------------------------------------------------ indexing
DEVI long pidx(const Geo &G, int L, int t, int k) { return G.off0 + ((long)t * L + k) * G.lev; }
#define AT(P, i, j) (P)[(long)(j) * G.pitch + (i)]

DEVI int stx_(int st) { return (st == SC || st == SY) ? 1 : 0; }
DEVI int sty_(int st) { return (st == SC || st == SX) ? 1 : 0; }
DEVI int floor2(int a) { return a >= 0 ? (a >> 1) : -((1 - a) >> 1); }

DEVI bool in_corner(const Geo &G, int st, int i, int j)
{
    int x2 = 2 * i + stx_(st), y2 = 2 * j + sty_(st), n2 = 2 * G.n;
    return G.cube && (x2 < 0 || x2 > n2) && (y2 < 0 || y2 > n2);
}

// Corner view: the edge-halo point a corner-block point (i, j) of stagger st
// reads in sweep mode `mode` (0 x, 1 y); cw reports the rotation sense.
DEVI void corner_src(const Geo &G, int st, int i, int j, int mode, int &qi, int &qj, bool &cw)
{
    int n2 = 2 * G.n;
    int x2 = 2 * i + stx_(st), y2 = 2 * j + sty_(st);
    int vx = x2 < 0 ? 0 : n2, vy = y2 < 0 ? 0 : n2;
    int c = (x2 < 0 ? 0 : 1) + (y2 < 0 ? 0 : 2);
    cw = mode == 0 ? (c == 0 || c == 3) : (c == 1 || c == 2);
    int dx = x2 - vx, dy = y2 - vy;
    int qx2 = cw ? vx + dy : vx - dy;
    int qy2 = cw ? vy - dx : vy + dx;
    qi = floor2(qx2);
    qj = floor2(qy2);
}

// scalar read through the corner view
template <class T>
DEVI T sv(const Geo &G, const T *P, int st, int i, int j, int mode)
{
    if (in_corner(G, st, i, j)) {
        int qi, qj;
        bool cw;
        corner_src(G, st, i, j, mode, qi, qj, cw);
        return AT(P, qi, qj);
    }
    return AT(P, i, j);
}
// x component of a pair (X at stagger stx, Y its partner) through the view;
// sgn = false for unsigned pairs (lengths)
template <class T>
DEVI T pvx(const Geo &G, const T *X, const T *Y, int stx, int i, int j, int mode, bool sgn)
{
    if (in_corner(G, stx, i, j)) {
        int qi, qj;
        bool cw;
        corner_src(G, stx, i, j, mode, qi, qj, cw);
        T v = AT(Y, qi, qj);
        return (cw && sgn) ? -v : v;
    }
    return AT(X, i, j);
}
template <class T>
DEVI T pvy(const Geo &G, const T *X, const T *Y, int sty, int i, int j, int mode, bool sgn)
{
    if (in_corner(G, sty, i, j)) {
        int qi, qj;
        bool cw;
        corner_src(G, sty, i, j, mode, qi, qj, cw);
        T v = AT(X, qi, qj);
        return (!cw && sgn) ? -v : v;
    }
    return AT(Y, i, j);
}

DEVI bool is_vertex(const Geo &G, int i, int j)
{
    return G.cube && (i == 0 || i == G.n) && (j == 0 || j == G.n);
}

#define KBEGIN(L)                                                    \
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);      \
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);      \
    if (i > ihi || j > jhi) return;                                  \
    int t = (int)blockIdx.z / (L), k = (int)blockIdx.z % (L);        \
    (void)t; (void)k;

#define KARGS int ilo, int ihi, int jlo, int jhi

struct Met {
    const double *m[M_COUNT];
};

// plane pointer of a 2-D metric for tile t
#define MP(name) (M.m[name] + G.off0 + (long)t * G.lev)

// ---------------------------------------------------------- launch timing
struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};
static struct {
    bool on = false;
    std::string filter;
    std::vector<TimingRec> recs;
} g_timing;

static bool timing_wanted(const char *name)
{
    return g_timing.on && std::strstr(name, g_timing.filter.c_str()) != nullptr;
}
static void timing_begin(const char *name, hipStream_t st, TimingRec &r)
{
    r.name = name;
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, st);
}
static void timing_end(hipStream_t st, TimingRec &r)
{
    (void)hipEventRecord(r.b, st);
    g_timing.recs.push_back(r);
}

template <class Kern, class... Args>
static void launch2d_named(const char *name, Kern kern, int ilo, int ihi, int jlo, int jhi, int planes,
                           hipStream_t st, Args... args)
{
    dim3 blk(64, 4, 1);
    dim3 grd((unsigned)((ihi - ilo + 64) / 64), (unsigned)((jhi - jlo + 4) / 4), (unsigned)planes);
    bool tm = timing_wanted(name);
    TimingRec r;
    if (tm) timing_begin(name, st, r);
    hipLaunchKernelGGL(kern, grd, blk, 0, st, ilo, ihi, jlo, jhi, args...);
    if (tm) timing_end(st, r);
}
#define launch2d(kern, ...) launch2d_named(#kern, kern, __VA_ARGS__)

// ====================================================================
// 1-D PPM face value (monotone): face between cells m-1 and m along a
// sweep, cell values q[0..5] = cells m-3..m+2, Courant number c.  Limited
// slope per cell (zero at extrema), fourth-order edge values, edge
// deviations clipped to twice the slope, mean of the parabola over the
// swept part of the upwind cell.
// ====================================================================
template <class T>
DEVI T lslope(T a, T b, T c)
{
    T d = (c - a) * (T)0.25;
    T mx = fmax(a, fmax(b, c)), mn = fmin(a, fmin(b, c));
    T lim = fmin(fabs(d), fmin(mx - b, b - mn));
    return d > 0 ? lim : (d < 0 ? -lim : (T)0);
}
template <class T>
DEVI T sgnT(T x) { return x > 0 ? (T)1 : (x < 0 ? (T)-1 : (T)0); }

template <class T>
DEVI T ppm6(T q0, T q1, T q2, T q3, T q4, T q5, T c)
{
    // cells m-3 .. m+2 -> q0 .. q5
    T d1 = lslope(q0, q1, q2), d2 = lslope(q1, q2, q3), d3 = lslope(q2, q3, q4),
      d4 = lslope(q3, q4, q5);
    const T third = (T)1 / (T)3;
    if (c > 0) {
        // upwind cell m-1 (q2): left edge between q1,q2, right edge between q2,q3
        T al = (T)0.5 * (q1 + q2) + (d1 - d2) * third;
        T ar = (T)0.5 * (q2 + q3) + (d2 - d3) * third;
        T s = sgnT(d2), a2 = (T)2 * fabs(d2);
        T bl = -s * fmin(a2, fabs(al - q2));
        T br = s * fmin(a2, fabs(ar - q2));
        return q2 + ((T)1 - c) * (br - c * (bl + br));
    } else {
        T al = (T)0.5 * (q2 + q3) + (d2 - d3) * third;
        T ar = (T)0.5 * (q3 + q4) + (d3 - d4) * third;
        T s = sgnT(d3), a2 = (T)2 * fabs(d3);
        T bl = -s * fmin(a2, fabs(al - q3));
        T br = s * fmin(a2, fabs(ar - q3));
        return q3 + ((T)1 + c) * (bl + c * (bl + br));
    }
}

// ====================================================================
// Halo exchange: plan-driven copies from the neighbour tile's interior
// (orientation transform folded into the plan for vector pairs).
// ====================================================================
template <class T>
__global__ void k_halo_scalar(Geo G, const HaloEnt *__restrict__ plan, int count, T *f, int L)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    int k = blockIdx.y;
    HaloEnt h = plan[e];
    f[pidx(G, L, h.dt, k) + h.di] = f[pidx(G, L, h.st, k) + h.si];
}

template <class T>
__global__ void k_halo_pair(Geo G, const HaloEnt *__restrict__ plan, int count, T *fx, T *fy, int L)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    int k = blockIdx.y;
    HaloEnt h = plan[e];
    const T *src = (h.sel & 1) ? fy : fx;
    T *dst = (h.sel & 4) ? fy : fx;
    T v = src[pidx(G, L, h.st, k) + h.si];
    dst[pidx(G, L, h.dt, k) + h.di] = (h.sel & 2) ? -v : v;
}

template <class T>
static void halo_scalar(const fv3_grid *g, T *f, int L, hipStream_t st)
{
    if (g->planC.count == 0) return;
    dim3 grd((g->planC.count + 255) / 256, L);
    bool tm = timing_wanted("k_halo_scalar");
    TimingRec r;
    if (tm) timing_begin("k_halo_scalar", st, r);
    hipLaunchKernelGGL(k_halo_scalar<T>, grd, dim3(256), 0, st, g->geo, g->planC.d, g->planC.count, f, L);
    if (tm) timing_end(st, r);
}
template <class T>
static void halo_pair(const fv3_grid *g, const Plan &p, T *fx, T *fy, int L, hipStream_t st)
{
    if (p.count == 0) return;
    dim3 grd((p.count + 255) / 256, L);
    bool tm = timing_wanted("k_halo_pair");
    TimingRec r;
    if (tm) timing_begin("k_halo_pair", st, r);
    hipLaunchKernelGGL(k_halo_pair<T>, grd, dim3(256), 0, st, g->geo, p.d, p.count, fx, fy, L);
    if (tm) timing_end(st, r);
}

// ====================================================================
// c_sw (half step dt2 on one level): D -> A -> C interpolation, upwind
// half-step cell fluxes, kinetic energy, corner vorticity, C-grid winds.
// ====================================================================
// A-grid winds at cells: u interpolated along y ((-1,9,9,-1)/16, y-sweep
// corner view), v along x (x-sweep view).
__global__ void k_csw_agrid(KARGS, Geo G, const B *u, const B *v, B *ua, B *va)
{
    KBEGIN(G.nz);
    if (in_corner(G, SC, i, j)) return;
    long o = pidx(G, G.nz, t, k);
    const B *U = u + o, *V = v + o;
    if (j >= -2 && j <= G.n + 1) {
        B a = pvx(G, U, V, SY, i, j - 1, 1, true), b = pvx(G, U, V, SY, i, j, 1, true),
          c = pvx(G, U, V, SY, i, j + 1, 1, true), d = pvx(G, U, V, SY, i, j + 2, 1, true);
        AT(ua + o, i, j) = (-a + 9.0 * b + 9.0 * c - d) / 16.0;
    }
    if (i >= -2 && i <= G.n + 1) {
        B a = pvy(G, U, V, SX, i - 1, j, 0, true), b = pvy(G, U, V, SX, i, j, 0, true),
          c = pvy(G, U, V, SX, i + 1, j, 0, true), d = pvy(G, U, V, SX, i + 2, j, 0, true);
        AT(va + o, i, j) = (-a + 9.0 * b + 9.0 * c - d) / 16.0;
    }
}

// C-grid winds before the update, normal-wind area fluxes over dt2 and the
// first-order upwind fluxes of delp, pt*delp, w*delp on the faces around the
// half-step cells (-1..n in both directions, without the four corner cells).
__global__ void k_csw_faces(KARGS, Geo G, Met M, B dt2, const B *u, const B *v, const B *delp,
                            const B *pt, const B *w, const B *ua, const B *va, B *ucp, B *vcp,
                            B *ax, B *ay, B *Fm, B *Fp, B *Fw, B *Gm, B *Gp, B *Gw)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const B *UA = ua + o, *VA = va + o, *D = delp + o, *PT = pt + o, *W = w + o;
    bool xf = (j >= -1 && j <= n) && ((j >= 0 && j < n) ? (i >= -1 && i <= n + 1) : (i >= 0 && i <= n));
    bool yf = (i >= -1 && i <= n) && ((i >= 0 && i < n) ? (j >= -1 && j <= n + 1) : (j >= 0 && j <= n));
    if (xf) {
        B a = pvx(G, UA, VA, SC, i - 2, j, 0, true), b = pvx(G, UA, VA, SC, i - 1, j, 0, true),
          c = pvx(G, UA, VA, SC, i, j, 0, true), d = pvx(G, UA, VA, SC, i + 1, j, 0, true);
        B uc0 = (-a + 9.0 * b + 9.0 * c - d) / 16.0;
        B fl = dt2 * (uc0 - AT(v + o, i, j) * AT(MP(M_COS_U), i, j)) / AT(MP(M_SIN_U), i, j) *
               AT(MP(M_DY), i, j);
        int up = fl > 0 ? i - 1 : i;
        B fm = fl * sv(G, D, SC, up, j, 0);
        AT(ucp + o, i, j) = uc0;
        AT(ax + o, i, j) = fl;
        AT(Fm + o, i, j) = fm;
        AT(Fp + o, i, j) = fm * sv(G, PT, SC, up, j, 0);
        AT(Fw + o, i, j) = fm * sv(G, W, SC, up, j, 0);
    }
    if (yf) {
        B a = pvy(G, UA, VA, SC, i, j - 2, 1, true), b = pvy(G, UA, VA, SC, i, j - 1, 1, true),
          c = pvy(G, UA, VA, SC, i, j, 1, true), d = pvy(G, UA, VA, SC, i, j + 1, 1, true);
        B vc0 = (-a + 9.0 * b + 9.0 * c - d) / 16.0;
        B fl = dt2 * (vc0 - AT(u + o, i, j) * AT(MP(M_COS_V), i, j)) / AT(MP(M_SIN_V), i, j) *
               AT(MP(M_DX), i, j);
        int up = fl > 0 ? j - 1 : j;
        B gm = fl * sv(G, D, SC, i, up, 1);
        AT(vcp + o, i, j) = vc0;
        AT(ay + o, i, j) = fl;
        AT(Gm + o, i, j) = gm;
        AT(Gp + o, i, j) = gm * sv(G, PT, SC, i, up, 1);
        AT(Gw + o, i, j) = gm * sv(G, W, SC, i, up, 1);
    }
}

// Half-step cell values and kinetic energy on the cross of cells -1..n;
// absolute vorticity on the corners 0..n (C-grid circulation; at a cube
// vertex the two faces next to the missing corner cell each count half).
__global__ void k_csw_cells(KARGS, Geo G, Met M, B dt2, const B *delp, const B *pt, const B *w,
                            const B *ua, const B *va, const B *ucp, const B *vcp, const B *Fm,
                            const B *Fp, const B *Fw, const B *Gm, const B *Gp, const B *Gw,
                            B *delpc, B *ptc, B *wc, B *ke, B *vort)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    bool cross = (i >= 0 && i < n) || (j >= 0 && j < n);
    if (cross) {
        B ar = AT(MP(M_AREA), i, j);
        B dp = AT(delp + o, i, j);
        B dc = dp + (AT(Fm + o, i, j) - AT(Fm + o, i + 1, j) + AT(Gm + o, i, j) - AT(Gm + o, i, j + 1)) / ar;
        AT(delpc + o, i, j) = dc;
        AT(ptc + o, i, j) =
            (AT(pt + o, i, j) * dp + (AT(Fp + o, i, j) - AT(Fp + o, i + 1, j) + AT(Gp + o, i, j) - AT(Gp + o, i, j + 1)) / ar) / dc;
        AT(wc + o, i, j) =
            (AT(w + o, i, j) * dp + (AT(Fw + o, i, j) - AT(Fw + o, i + 1, j) + AT(Gw + o, i, j) - AT(Gw + o, i, j + 1)) / ar) / dc;
        B sa = AT(MP(M_SIN_A), i, j), ca = AT(MP(M_COS_A), i, j);
        B s2 = sa * sa;
        B a = AT(ua + o, i, j), b = AT(va + o, i, j);
        B uu = (a - b * ca) / s2, vv = (b - a * ca) / s2;
        AT(ke + o, i, j) = 0.5 * dt2 *
                           (uu * (uu > 0 ? AT(ucp + o, i, j) : AT(ucp + o, i + 1, j)) +
                            vv * (vv > 0 ? AT(vcp + o, i, j) : AT(vcp + o, i, j + 1)));
    }
    if (i >= 0 && i <= n && j >= 0 && j <= n) {
        B ws = 1, wn = 1, ww = 1, we = 1;
        if (is_vertex(G, i, j)) {
            if (j == 0) ws = 0.5; else wn = 0.5;
            if (i == 0) ww = 0.5; else we = 0.5;
        }
        B circ = ws * AT(ucp + o, i, j - 1) * AT(MP(M_DXC), i, j - 1) -
                 wn * AT(ucp + o, i, j) * AT(MP(M_DXC), i, j) -
                 ww * AT(vcp + o, i - 1, j) * AT(MP(M_DYC), i - 1, j) +
                 we * AT(vcp + o, i, j) * AT(MP(M_DYC), i, j);
        AT(vort + o, i, j) = AT(MP(M_FB), i, j) + circ / AT(MP(M_AREA_C), i, j);
    }
}

// C-grid wind update on the interior faces: upwinded vorticity flux plus
// kinetic-energy gradient.
__global__ void k_csw_update(KARGS, Geo G, Met M, B dt2, const B *u, const B *v, const B *ucp,
                             const B *vcp, const B *ke, const B *vort, B *uc, B *vc)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    if (j < n) {
        B u0 = AT(ucp + o, i, j);
        B fy1 = dt2 * (AT(v + o, i, j) - u0 * AT(MP(M_COS_U), i, j)) / AT(MP(M_SIN_U), i, j);
        B vt = fy1 > 0 ? AT(vort + o, i, j) : AT(vort + o, i, j + 1);
        AT(uc + o, i, j) = u0 + fy1 * vt + (AT(ke + o, i - 1, j) - AT(ke + o, i, j)) / AT(MP(M_DXC), i, j);
    }
    if (i < n) {
        B v0 = AT(vcp + o, i, j);
        B fx1 = dt2 * (AT(u + o, i, j) - v0 * AT(MP(M_COS_V), i, j)) / AT(MP(M_SIN_V), i, j);
        B vt = fx1 > 0 ? AT(vort + o, i, j) : AT(vort + o, i + 1, j);
        AT(vc + o, i, j) = v0 - fx1 * vt + (AT(ke + o, i, j - 1) - AT(ke + o, i, j)) / AT(MP(M_DYC), i, j);
    }
}

// ====================================================================
// Vertical column work (one thread per column, k marching in FP64).
// ====================================================================
DEVI double zs_at(const Geo &G, const double *phis, int t, int i, int j, int mode)
{
    if (!phis) return 0.0;
    const double *P = phis + pidx(G, 1, t, 0);
    return sv(G, P, SC, i, j, mode) / GRAV;
}

// dz_c: half-step interface heights by first-order upwind transport of the
// interface heights with layer-averaged area fluxes (top interface: top
// layer), advective form, surface fixed; output the half-step thicknesses.
__global__ void k_dzc(KARGS, Geo G, Met M, const double *delz, const double *phis, const B *ax,
                      const B *ay, double *delzc)
{
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (i > ihi || j > jhi) return;
    int n = G.n, nz = G.nz, t = blockIdx.z;
    if (!((i >= 0 && i < n) || (j >= 0 && j < n))) return;
    double area = AT(MP(M_AREA), i, j);
    double zc = zs_at(G, phis, t, i, j, 0);
    double zw = zs_at(G, phis, t, i - 1, j, 0), ze = zs_at(G, phis, t, i + 1, j, 0);
    double zsou = zs_at(G, phis, t, i, j - 1, 1), znor = zs_at(G, phis, t, i, j + 1, 1);
    double zsurf = zc;
    double zprev = zsurf;   // new height of the interface below
    for (int K = nz - 1; K >= 0; K--) {
        long o = pidx(G, nz, t, K);
        const double *D = delz + o;
        zc -= AT(D, i, j);
        zw -= sv(G, D, SC, i - 1, j, 0);
        ze -= sv(G, D, SC, i + 1, j, 0);
        zsou -= sv(G, D, SC, i, j - 1, 1);
        znor -= sv(G, D, SC, i, j + 1, 1);
        long ob = K > 0 ? pidx(G, nz, t, K - 1) : o;
        double a0 = K == 0 ? (double)AT(ax + o, i, j) : 0.5 * ((double)AT(ax + ob, i, j) + (double)AT(ax + o, i, j));
        double a1 = K == 0 ? (double)AT(ax + o, i + 1, j) : 0.5 * ((double)AT(ax + ob, i + 1, j) + (double)AT(ax + o, i + 1, j));
        double b0 = K == 0 ? (double)AT(ay + o, i, j) : 0.5 * ((double)AT(ay + ob, i, j) + (double)AT(ay + o, i, j));
        double b1 = K == 0 ? (double)AT(ay + o, i, j + 1) : 0.5 * ((double)AT(ay + ob, i, j + 1) + (double)AT(ay + o, i, j + 1));
        double z0 = a0 > 0 ? zw : zc, z1 = a1 > 0 ? zc : ze;
        double y0 = b0 > 0 ? zsou : zc, y1 = b1 > 0 ? zc : znor;
        double zn = (zc * area + a0 * z0 - a1 * z1 + b0 * y0 - b1 * y1) / (area + a0 - a1 + b0 - b1);
        AT(delzc + o, i, j) = zprev - zn;
        zprev = zn;
    }
}

// Semi-implicit column solve (riem_solver_c / riem_solver3, Sec. IX-B):
// hydrostatic interface pressure from delp (top down), nonhydrostatic
// pressure from the equation of state, mass-weighted interface perturbation,
// backward-Euler tridiagonal system in w (Thomas, positive pivots), new
// perturbation by a top-down scan, thickness by inverting the equation of
// state, heights by a bottom-up scan.  Temporaries in FP64 scratch columns.
template <class TW>
__global__ void k_sim1(KARGS, Geo G, double dt, double ptop, const B *dpi, const B *theta,
                       const double *delz, const TW *w, const double *phis, double *cpv,
                       double *dpv, double *wnv, TW *w_out, double *delz_out, double *pfull,
                       double *phi, int need_cross)
{
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (i > ihi || j > jhi) return;
    int n = G.n, nz = G.nz, t = blockIdx.z;
    if (need_cross && !((i >= 0 && i < n) || (j >= 0 && j < n))) return;
    const double kap = RDGAS / CP_AIR, gam = 1.0 / (1.0 - kap), rgam = 1.0 - kap;
    long cidx = (long)j * G.pitch + i;
    auto L = [&](int k) { return pidx(G, nz, t, k) + cidx; };
    auto LI = [&](int K) { return pidx(G, nz + 1, t, K) + cidx; };
    // forward sweep with a one-layer look-ahead
    double pi_k = ptop;                 // interface k
    double dp0 = (double)dpi[L(0)];
    double pi_k1 = pi_k + dp0;
    double m0 = dp0 / GRAV, h0 = -delz[L(0)];
    double pib0 = dp0 / (log(pi_k1) - log(pi_k));
    double pp0 = P_REF * pow(RDGAS * (double)theta[L(0)] * m0 / (h0 * P_REF), gam) - pib0;
    double pps_k = 0.0, A_k = 0.0;      // at interface k
    double cprev = 0.0, dprev = 0.0;
    for (int k = 0; k < nz; k++) {
        double pps_k1, A_k1;
        double m1 = 0, h1 = 0, pp1 = 0, dp1 = 0, pi_k2 = 0;
        if (k < nz - 1) {
            dp1 = (double)dpi[L(k + 1)];
            pi_k2 = pi_k1 + dp1;
            m1 = dp1 / GRAV;
            h1 = -delz[L(k + 1)];
            double pib1 = dp1 / (log(pi_k2) - log(pi_k1));
            pp1 = P_REF * pow(RDGAS * (double)theta[L(k + 1)] * m1 / (h1 * P_REF), gam) - pib1;
            pps_k1 = (dp1 * pp0 + dp0 * pp1) / (dp0 + dp1);
            A_k1 = gam * (pi_k1 + pps_k1) * dt * dt / (0.5 * (h0 + h1));
        } else {
            pps_k1 = pp0;
            A_k1 = gam * (pi_k1 + pps_k1) * dt * dt / (0.5 * h0);
        }
        double lower = k > 0 ? -A_k : 0.0;
        double diag = m0 + A_k + A_k1;
        double upper = k < nz - 1 ? -A_k1 : 0.0;
        double rhs = m0 * (double)w[L(k)] + dt * (pps_k1 - pps_k);
        double piv = diag - lower * cprev;
        double ck = upper / piv;
        double dk = (rhs - lower * dprev) / piv;
        cpv[L(k)] = ck;
        dpv[L(k)] = dk;
        cprev = ck;
        dprev = dk;
        // advance
        pi_k = pi_k1; pi_k1 = pi_k2; dp0 = dp1; m0 = m1; h0 = h1; pp0 = pp1;
        pps_k = pps_k1; A_k = A_k1;
    }
    // back substitution
    double wn = 0.0;
    for (int k = nz - 1; k >= 0; k--) {
        wn = dpv[L(k)] - cpv[L(k)] * wn;
        wnv[L(k)] = wn;
    }
    // new perturbation (top down) and thicknesses
    double ppn = 0.0, pik = ptop;
    if (pfull) pfull[LI(0)] = ptop;
    for (int k = 0; k < nz; k++) {
        double dp = (double)dpi[L(k)];
        double m = dp / GRAV;
        double pik1 = pik + dp;
        double pib = dp / (log(pik1) - log(pik));
        double wk = wnv[L(k)];
        double ppn1 = ppn + m * (wk - (double)w[L(k)]) / dt;
        double pn = pib + 0.5 * (ppn + ppn1);
        double hn = RDGAS * (double)theta[L(k)] * m / P_REF * pow(P_REF / pn, rgam);
        cpv[L(k)] = hn;   // reuse as the new thickness
        if (pfull) pfull[LI(k + 1)] = pik1 + ppn1;
        if (w_out) w_out[L(k)] = (TW)wk;
        ppn = ppn1;
        pik = pik1;
    }
    double z = phis ? phis[pidx(G, 1, t, 0) + cidx] / GRAV : 0.0;
    if (phi) phi[LI(nz)] = GRAV * z;
    for (int k = nz - 1; k >= 0; k--) {
        double hn = cpv[L(k)];
        z += hn;
        if (phi) phi[LI(k)] = GRAV * z;
        if (delz_out) delz_out[L(k)] = -hn;
    }
}

// Finite-volume pressure gradient between two columns W, E over one layer:
// contour integral of p dPhi around the quadrilateral of the two columns'
// interfaces k, k+1, over the mean layer mass and the distance L.
DEVI double pgf(double dt, double L, double dW, double dE, double zW0, double zW1, double zE0,
                double zE1, double pW0, double pW1, double pE0, double pE1)
{
    return dt / (L * (dW + dE)) * ((zW1 - zE0) * (pE1 - pW0) + (zW0 - zE1) * (pW1 - pE0));
}

// p_grad_c on the interior C-grid faces with the half-step cells' pressure
// and geopotential; layer mass weights from delpc.
__global__ void k_pgradc(KARGS, Geo G, Met M, double dt2, const B *delpc, const double *pkc,
                         const double *gz, B *uc, B *vc)
{
    KBEGIN(G.nz);
    int n = G.n, nz = G.nz;
    long o = pidx(G, nz, t, k), o0 = pidx(G, nz + 1, t, k), o1 = pidx(G, nz + 1, t, k + 1);
    const B *D = delpc + o;
    if (j < n) {
        int iw = i - 1, ie = i;
        AT(uc + o, i, j) += (B)pgf(dt2, AT(MP(M_DXC), i, j), AT(D, iw, j), AT(D, ie, j), AT(gz + o0, iw, j),
                                   AT(gz + o1, iw, j), AT(gz + o0, ie, j), AT(gz + o1, ie, j), AT(pkc + o0, iw, j),
                                   AT(pkc + o1, iw, j), AT(pkc + o0, ie, j), AT(pkc + o1, ie, j));
    }
    if (i < n) {
        int js = j - 1, jn = j;
        AT(vc + o, i, j) += (B)pgf(dt2, AT(MP(M_DYC), i, j), AT(D, i, js), AT(D, i, jn), AT(gz + o0, i, js),
                                   AT(gz + o1, i, js), AT(gz + o0, i, jn), AT(gz + o1, i, jn), AT(pkc + o0, i, js),
                                   AT(pkc + o1, i, js), AT(pkc + o0, i, jn), AT(pkc + o1, i, jn));
    }
}

// ====================================================================
// fv_tp_2d (Sec. IX-C): Lin-Rood flux-form transport on one level.
// Three passes: outer PPM fluxes of q in both directions; inner advective
// half updates; PPM fluxes of the cross-updated fields and the averaged,
// weighted fluxes.  q has Lq levels, the Courant/area-flux arrays Lc; plane
// k of q pairs with plane k of the fluxes.
// ====================================================================
template <class T>
__global__ void k_fv_outer(KARGS, Geo G, int Lq, int Lc, const T *q, const B *crx, const B *cry,
                           T *fx2, T *fy2)
{
    KBEGIN(Lc);
    int n = G.n;
    const T *Q = q + pidx(G, Lq, t, k);
    long oc = pidx(G, Lc, t, k);
    if (i >= -3 && i <= n + 2 && j >= 0 && j <= n) {
        T c = (T)AT(cry + oc, i, j);
        AT(fy2 + oc, i, j) = ppm6(sv(G, Q, SC, i, j - 3, 1), sv(G, Q, SC, i, j - 2, 1), sv(G, Q, SC, i, j - 1, 1),
                                  sv(G, Q, SC, i, j, 1), sv(G, Q, SC, i, j + 1, 1), sv(G, Q, SC, i, j + 2, 1), c);
    }
    if (i >= 0 && i <= n && j >= -3 && j <= n + 2) {
        T c = (T)AT(crx + oc, i, j);
        AT(fx2 + oc, i, j) = ppm6(sv(G, Q, SC, i - 3, j, 0), sv(G, Q, SC, i - 2, j, 0), sv(G, Q, SC, i - 1, j, 0),
                                  sv(G, Q, SC, i, j, 0), sv(G, Q, SC, i + 1, j, 0), sv(G, Q, SC, i + 2, j, 0), c);
    }
}

template <class T>
__global__ void k_fv_inner(KARGS, Geo G, Met M, int Lq, int Lc, const T *q, const B *xfx,
                           const B *yfx, const T *fx2, const T *fy2, T *qi, T *qj)
{
    KBEGIN(Lc);
    int n = G.n;
    const T *Q = q + pidx(G, Lq, t, k);
    long oc = pidx(G, Lc, t, k);
    T ar = (T)AT(MP(M_AREA), i, j);
    if (i >= -3 && i <= n + 2 && j >= 0 && j < n) {
        T y0 = (T)AT(yfx + oc, i, j), y1 = (T)AT(yfx + oc, i, j + 1);
        AT(qi + oc, i, j) = (AT(Q, i, j) * ar + y0 * AT(fy2 + oc, i, j) - y1 * AT(fy2 + oc, i, j + 1)) / (ar + y0 - y1);
    }
    if (i >= 0 && i < n && j >= -3 && j <= n + 2) {
        T x0 = (T)AT(xfx + oc, i, j), x1 = (T)AT(xfx + oc, i + 1, j);
        AT(qj + oc, i, j) = (AT(Q, i, j) * ar + x0 * AT(fx2 + oc, i, j) - x1 * AT(fx2 + oc, i + 1, j)) / (ar + x0 - x1);
    }
}

template <class T, class TM>
__global__ void k_fv_flux(KARGS, Geo G, int Lc, const B *crx, const B *cry, const B *xfx,
                          const B *yfx, const TM *mx, const TM *my, const T *fx2, const T *fy2,
                          const T *qi, const T *qj, T *FX, T *FY)
{
    KBEGIN(Lc);
    int n = G.n;
    long oc = pidx(G, Lc, t, k);
    if (i >= 0 && i <= n && j >= 0 && j < n) {
        const T *P = qi + oc;
        T fx = ppm6(AT(P, i - 3, j), AT(P, i - 2, j), AT(P, i - 1, j), AT(P, i, j), AT(P, i + 1, j), AT(P, i + 2, j),
                    (T)AT(crx + oc, i, j));
        T wgt = mx ? (T)AT(mx + oc, i, j) : (T)AT(xfx + oc, i, j);
        AT(FX + oc, i, j) = (T)0.5 * (fx + AT(fx2 + oc, i, j)) * wgt;
    }
    if (i >= 0 && i < n && j >= 0 && j <= n) {
        const T *P = qj + oc;
        T fy = ppm6(AT(P, i, j - 3), AT(P, i, j - 2), AT(P, i, j - 1), AT(P, i, j), AT(P, i, j + 1), AT(P, i, j + 2),
                    (T)AT(cry + oc, i, j));
        T wgt = my ? (T)AT(my + oc, i, j) : (T)AT(yfx + oc, i, j);
        AT(FY + oc, i, j) = (T)0.5 * (fy + AT(fy2 + oc, i, j)) * wgt;
    }
}

struct FvTmp {
    void *fx2, *fy2, *qi, *qj;
};

template <class T, class TM>
static void fv_tp_2d(const fv3_grid *g, Met M, int Lq, int Lc, int planes, const T *q, const B *crx,
                     const B *cry, const B *xfx, const B *yfx, const TM *mx, const TM *my, T *FX,
                     T *FY, FvTmp tmp, hipStream_t st)
{
    int n = g->n;
    const Geo &G = g->geo;
    T *fx2 = (T *)tmp.fx2, *fy2 = (T *)tmp.fy2, *qi = (T *)tmp.qi, *qj = (T *)tmp.qj;
    launch2d(k_fv_outer<T>, -3, n + 2, -3, n + 2, planes, st, G, Lq, Lc, q, crx, cry, fx2, fy2);
    launch2d(k_fv_inner<T>, -3, n + 2, -3, n + 2, planes, st, G, M, Lq, Lc, q, xfx, yfx,
             (const T *)fx2, (const T *)fy2, qi, qj);
    launch2d(k_fv_flux<T, TM>, 0, n, 0, n, planes, st, G, Lc, crx, cry, xfx, yfx, mx, my,
             (const T *)fx2, (const T *)fy2, (const T *)qi, (const T *)qj, FX, FY);
}

// ====================================================================
// d_sw (full step bdt on one level)
// ====================================================================
// Courant numbers and area fluxes from the contravariant half-step C-grid
// winds (partner component: four-point mean of the other C-grid wind).
__global__ void k_dsw_courant(KARGS, Geo G, Met M, B bdt, const B *uc, const B *vc, B *ut, B *vt,
                              B *crx, B *cry, B *xfx, B *yfx, int *flags)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const B *UC = uc + o, *VC = vc + o;
    const double *dxa = MP(M_DXA), *dya = MP(M_DYA);
    bool bad = false;
    if (i >= 0 && i <= n && j >= -3 && j <= n + 2) {
        B vb = 0.25 * (pvy(G, UC, VC, SY, i - 1, j, 0, true) + pvy(G, UC, VC, SY, i, j, 0, true) +
                       pvy(G, UC, VC, SY, i - 1, j + 1, 0, true) + pvy(G, UC, VC, SY, i, j + 1, 0, true));
        B su = AT(MP(M_SIN_U), i, j);
        B uu = (AT(UC, i, j) - vb * AT(MP(M_COS_U), i, j)) / (su * su);
        int up = uu > 0 ? i - 1 : i;
        B cr = bdt * uu / pvx(G, dxa, dya, SC, up, j, 0, false);
        AT(ut + o, i, j) = uu;
        AT(crx + o, i, j) = cr;
        AT(xfx + o, i, j) = bdt * uu * su * AT(MP(M_DY), i, j);
        bad |= fabs(cr) > 1.0;
    }
    if (i >= -3 && i <= n + 2 && j >= 0 && j <= n) {
        B ub = 0.25 * (pvx(G, UC, VC, SX, i, j - 1, 1, true) + pvx(G, UC, VC, SX, i + 1, j - 1, 1, true) +
                       pvx(G, UC, VC, SX, i, j, 1, true) + pvx(G, UC, VC, SX, i + 1, j, 1, true));
        B sv_ = AT(MP(M_SIN_V), i, j);
        B vv = (AT(VC, i, j) - ub * AT(MP(M_COS_V), i, j)) / (sv_ * sv_);
        int up = vv > 0 ? j - 1 : j;
        B cr = bdt * vv / pvy(G, dxa, dya, SC, i, up, 1, false);
        AT(vt + o, i, j) = vv;
        AT(cry + o, i, j) = cr;
        AT(yfx + o, i, j) = bdt * vv * sv_ * AT(MP(M_DX), i, j);
        bad |= fabs(cr) > 1.0;
    }
    if (bad) atomicOr(flags, 1);
}

// new delp from the mass fluxes; accumulate mass fluxes and Courant numbers
__global__ void k_dsw_mass(KARGS, Geo G, Met M, const B *delp, const B *FX, const B *FY,
                           const B *crx, const B *cry, B *dn, double *mfx, double *mfy, B *cx,
                           B *cy)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    if (i < n && j < n)
        AT(dn + o, i, j) = AT(delp + o, i, j) +
                           (AT(FX + o, i, j) - AT(FX + o, i + 1, j) + AT(FY + o, i, j) - AT(FY + o, i, j + 1)) /
                               AT(MP(M_AREA), i, j);
    if (j < n) {
        AT(mfx + o, i, j) += (double)AT(FX + o, i, j);
        AT(cx + o, i, j) += AT(crx + o, i, j);
    }
    if (i < n) {
        AT(mfy + o, i, j) += (double)AT(FY + o, i, j);
        AT(cy + o, i, j) += AT(cry + o, i, j);
    }
}

// mass-weighted update of a transported cell field (pt or w)
__global__ void k_dsw_scalar(KARGS, Geo G, Met M, const B *q, const B *delp, const B *dn,
                             const B *GX, const B *GY, B *qn)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    B ar = AT(MP(M_AREA), i, j);
    AT(qn + o, i, j) = (AT(q + o, i, j) * AT(delp + o, i, j) * ar + AT(GX + o, i, j) - AT(GX + o, i + 1, j) +
                        AT(GY + o, i, j) - AT(GY + o, i, j + 1)) /
                       (AT(dn + o, i, j) * ar);
}

// kinetic energy at corners: D-grid u upwinded along x and v along y by PPM
// with the corner displacements of the contravariant C-grid winds
__global__ void k_dsw_ke(KARGS, Geo G, Met M, B bdt, const B *u, const B *v, const B *ut,
                         const B *vt, B *ke)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    const B *U = u + o, *V = v + o;
    B ub = 0.5 * bdt * (AT(ut + o, i, j - 1) + AT(ut + o, i, j));
    B vb = 0.5 * bdt * (AT(vt + o, i - 1, j) + AT(vt + o, i, j));
    B cu = ub / AT(MP(M_DX), ub > 0 ? i - 1 : i, j);
    B cv = vb / AT(MP(M_DY), i, vb > 0 ? j - 1 : j);
    B uu = ppm6(AT(U, i - 3, j), AT(U, i - 2, j), AT(U, i - 1, j), AT(U, i, j), AT(U, i + 1, j), AT(U, i + 2, j), cu);
    B vv = ppm6(AT(V, i, j - 3), AT(V, i, j - 2), AT(V, i, j - 1), AT(V, i, j), AT(V, i, j + 1), AT(V, i, j + 2), cv);
    AT(ke + o, i, j) = 0.5 * (ub * uu + vb * vv);
}

// absolute vorticity at cells from the D-grid circulation
__global__ void k_dsw_omega(KARGS, Geo G, Met M, const B *u, const B *v, B *om)
{
    KBEGIN(G.nz);
    if (in_corner(G, SC, i, j)) return;
    long o = pidx(G, G.nz, t, k);
    const B *U = u + o, *V = v + o;
    const double *dx = MP(M_DX), *dy = MP(M_DY);
    AT(om + o, i, j) = AT(MP(M_FC), i, j) + (AT(U, i, j) * AT(dx, i, j) - AT(U, i, j + 1) * AT(dx, i, j + 1) -
                                             AT(V, i, j) * AT(dy, i, j) + AT(V, i + 1, j) * AT(dy, i + 1, j)) /
                                                AT(MP(M_AREA), i, j);
}

// D-grid wind update from kinetic-energy differences and vorticity fluxes;
// commit the transported delp, pt, w.
__global__ void k_dsw_update(KARGS, Geo G, Met M, const B *ke, const B *VX, const B *VY,
                             const B *dn, const B *pn, const B *wn, B *u, B *v, B *delp, B *pt, B *w)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const B *KE = ke + o;
    if (i < n) AT(u + o, i, j) = AT(u + o, i, j) + (AT(KE, i, j) - AT(KE, i + 1, j) + AT(VY + o, i, j)) / AT(MP(M_DX), i, j);
    if (j < n) AT(v + o, i, j) = AT(v + o, i, j) + (AT(KE, i, j) - AT(KE, i, j + 1) - AT(VX + o, i, j)) / AT(MP(M_DY), i, j);
    if (i < n && j < n) {
        AT(delp + o, i, j) = AT(dn + o, i, j);
        AT(pt + o, i, j) = AT(pn + o, i, j);
        AT(w + o, i, j) = AT(wn + o, i, j);
    }
}

// ====================================================================
// dz_d: interface heights transported by fv_tp_2d with layer-averaged
// Courant numbers and area fluxes, advective form, surface fixed.
// ====================================================================
__global__ void k_heights(KARGS, Geo G, const double *delz, const double *phis, double *zh)
{
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (i > ihi || j > jhi) return;
    int nz = G.nz, t = blockIdx.z;
    if (in_corner(G, SC, i, j)) return;
    long c = (long)j * G.pitch + i;
    double z = phis ? phis[pidx(G, 1, t, 0) + c] / GRAV : 0.0;
    zh[pidx(G, nz + 1, t, nz) + c] = z;
    for (int k = nz - 1; k >= 0; k--) {
        z -= delz[pidx(G, nz, t, k) + c];
        zh[pidx(G, nz + 1, t, k) + c] = z;
    }
}

__global__ void k_iface_flux(KARGS, Geo G, const B *crx, const B *cry, const B *xfx,
                             const B *yfx, B *cxI, B *cyI, B *xI, B *yI)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k), ob = pidx(G, G.nz, t, k > 0 ? k - 1 : 0);
    long c = (long)j * G.pitch + i;
    if (k == 0) {
        cxI[o + c] = crx[o + c]; cyI[o + c] = cry[o + c]; xI[o + c] = xfx[o + c]; yI[o + c] = yfx[o + c];
    } else {
        cxI[o + c] = 0.5 * (crx[ob + c] + crx[o + c]);
        cyI[o + c] = 0.5 * (cry[ob + c] + cry[o + c]);
        xI[o + c] = 0.5 * (xfx[ob + c] + xfx[o + c]);
        yI[o + c] = 0.5 * (yfx[ob + c] + yfx[o + c]);
    }
}

__global__ void k_zh_update(KARGS, Geo G, Met M, const double *zh, const double *ZX,
                            const double *ZY, const B *xI, const B *yI, double *zn)
{
    KBEGIN(G.nz);
    int nz = G.nz;
    long oq = pidx(G, nz + 1, t, k), oc = pidx(G, nz, t, k);
    double ar = AT(MP(M_AREA), i, j);
    AT(zn + oq, i, j) = (AT(zh + oq, i, j) * ar + AT(ZX + oc, i, j) - AT(ZX + oc, i + 1, j) + AT(ZY + oc, i, j) -
                         AT(ZY + oc, i, j + 1)) /
                        (ar + (double)AT(xI + oc, i, j) - (double)AT(xI + oc, i + 1, j) +
                         (double)AT(yI + oc, i, j) - (double)AT(yI + oc, i, j + 1));
}

__global__ void k_delz_from_zh(KARGS, Geo G, const double *zn, const double *phis, double *delz)
{
    KBEGIN(G.nz);
    int nz = G.nz;
    double below = k == nz - 1 ? (phis ? AT(phis + pidx(G, 1, t, 0), i, j) / GRAV : 0.0)
                               : AT(zn + pidx(G, nz + 1, t, k + 1), i, j);
    AT(delz + pidx(G, nz, t, k), i, j) = below - AT(zn + pidx(G, nz + 1, t, k), i, j);
}

// ====================================================================
// nh_p_grad: corner values by the fourth-order (-1,7,7,-1)/12 tensor
// interpolation (inner pass along x with the x-sweep corner view; mean of
// the three cells at a cube vertex) and the finite-volume pressure gradient
// along each D-grid edge.
// ====================================================================
template <class T>
__global__ void k_corner_interp(KARGS, Geo G, int L, const T *q, double *qB)
{
    KBEGIN(L);
    long o = pidx(G, L, t, k);
    const T *Q = q + o;
    double r;
    if (is_vertex(G, i, j)) {
        double s = 0.0;
        int ci[4] = {i - 1, i, i, i - 1}, cj[4] = {j - 1, j - 1, j, j};
        for (int c = 0; c < 4; c++)
            if (!in_corner(G, SC, ci[c], cj[c])) s += (double)AT(Q, ci[c], cj[c]);
        r = s / 3.0;
    } else {
        const double w4[4] = {-1.0 / 12.0, 7.0 / 12.0, 7.0 / 12.0, -1.0 / 12.0};
        r = 0.0;
        for (int b = 0; b < 4; b++) {
            double row = 0.0;
            for (int a = 0; a < 4; a++) row += w4[a] * (double)sv(G, Q, SC, i + a - 2, j + b - 2, 0);
            r += w4[b] * row;
        }
    }
    AT(qB + o, i, j) = r;
}

__global__ void k_nhpgrad(KARGS, Geo G, Met M, double bdt, const double *pB, const double *zB,
                          const double *dB, B *u, B *v)
{
    KBEGIN(G.nz);
    int n = G.n, nz = G.nz;
    long o = pidx(G, nz, t, k), o0 = pidx(G, nz + 1, t, k), o1 = pidx(G, nz + 1, t, k + 1);
    const double *P0 = pB + o0, *P1 = pB + o1, *Z0 = zB + o0, *Z1 = zB + o1, *D = dB + o;
    if (i < n)
        AT(u + o, i, j) += (B)pgf(bdt, AT(MP(M_DX), i, j), AT(D, i, j), AT(D, i + 1, j), AT(Z0, i, j), AT(Z1, i, j),
                                  AT(Z0, i + 1, j), AT(Z1, i + 1, j), AT(P0, i, j), AT(P1, i, j), AT(P0, i + 1, j),
                                  AT(P1, i + 1, j));
    if (j < n)
        AT(v + o, i, j) += (B)pgf(bdt, AT(MP(M_DY), i, j), AT(D, i, j), AT(D, i, j + 1), AT(Z0, i, j), AT(Z1, i, j),
                                  AT(Z0, i, j + 1), AT(Z1, i, j + 1), AT(P0, i, j), AT(P1, i, j), AT(P0, i, j + 1),
                                  AT(P1, i, j + 1));
}

// ====================================================================
// utilities: fills, copies, finiteness check, tracer helpers
// ====================================================================
template <class T>
__global__ void k_fill(T *p, long count, T val)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = val;
}
template <class TS, class TD>
__global__ void k_copy(const TS *s, TD *d, long count)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) d[e] = (TD)s[e];
}
template <class T>
static void fill(T *p, long count, T val, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, val);
}
template <class TS, class TD>
static void copy(const TS *s, TD *d, long count, hipStream_t st)
{
    hipLaunchKernelGGL((k_copy<TS, TD>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, s, d, count);
}

template <class T>
__global__ void k_check_finite(KARGS, Geo G, int L, const T *f, int *flags)
{
    KBEGIN(L);
    if (!isfinite((double)AT(f + pidx(G, L, t, k), i, j))) atomicOr(flags + 1, 1);
}

// tracer: area fluxes from the accumulated Courant numbers, scaled by 1/nsplt
__global__ void k_tracer_flux(KARGS, Geo G, Met M, double rs, const B *cx, const B *cy,
                              const double *mfx, const double *mfy, B *crs, B *crys, B *xfx,
                              B *yfx, double *mxs, double *mys)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const double *dxa = MP(M_DXA), *dya = MP(M_DYA);
    if (i >= 0 && i <= n && j >= -3 && j <= n + 2) {
        B c = AT(cx + o, i, j);
        int up = c > 0 ? i - 1 : i;
        AT(xfx + o, i, j) = (B)(c * pvx(G, dxa, dya, SC, up, j, 0, false) * AT(MP(M_DY), i, j) * AT(MP(M_SIN_U), i, j) / rs);
        AT(crs + o, i, j) = (B)(c / rs);
        AT(mxs + o, i, j) = AT(mfx + o, i, j) / rs;
    }
    if (i >= -3 && i <= n + 2 && j >= 0 && j <= n) {
        B c = AT(cy + o, i, j);
        int up = c > 0 ? j - 1 : j;
        AT(yfx + o, i, j) = (B)(c * pvy(G, dxa, dya, SC, i, up, 1, false) * AT(MP(M_DX), i, j) * AT(MP(M_SIN_V), i, j) / rs);
        AT(crys + o, i, j) = (B)(c / rs);
        AT(mys + o, i, j) = AT(mfy + o, i, j) / rs;
    }
}

__global__ void k_tracer_dp(KARGS, Geo G, Met M, const double *dp1, const double *mxs,
                            const double *mys, double *dp2)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    AT(dp2 + o, i, j) = AT(dp1 + o, i, j) + (AT(mxs + o, i, j) - AT(mxs + o, i + 1, j) + AT(mys + o, i, j) -
                                             AT(mys + o, i, j + 1)) /
                                                AT(MP(M_AREA), i, j);
}

__global__ void k_tracer_update(KARGS, Geo G, Met M, const double *dp1, const double *dp2,
                                const B *FX, const B *FY, B *q)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    double a = AT(MP(M_AREA), i, j);
    AT(q + o, i, j) = (B)(((double)AT(q + o, i, j) * AT(dp1 + o, i, j) * a + (double)AT(FX + o, i, j) -
                           (double)AT(FX + o, i + 1, j) + (double)AT(FY + o, i, j) - (double)AT(FY + o, i, j + 1)) /
                          (AT(dp2 + o, i, j) * a));
}

__global__ void k_absmax(KARGS, Geo G, const B *cx, const B *cy, unsigned long long *out)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    double m = 0.0;
    if (j < n) m = fmax(m, fabs((double)AT(cx + o, i, j)));
    if (i < n) m = fmax(m, fabs((double)AT(cy + o, i, j)));
    // non-negative doubles order like their bit patterns
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Neumaier-compensated sums: each thread sums its column over levels in a
// fixed order, then the block reduces pairs (s, c) exactly as Neumaier
// additions, one partial per block; the host adds the partials in order.
DEVI void neu_add(double &s, double &c, double x)
{
    double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

__global__ void k_mass_partial(KARGS, Geo G, Met M, const B *delp, const B *pt, const B *q,
                               int which, double *part)
{
    __shared__ double ss[256], sc[256];
    int tid = threadIdx.y * blockDim.x + threadIdx.x;
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    int t = blockIdx.z;
    double s = 0.0, c = 0.0;
    if (i <= ihi && j <= jhi) {
        double ar = AT(MP(M_AREA), i, j);
        for (int k = 0; k < G.nz; k++) {
            long o = pidx(G, G.nz, t, k);
            double m = (double)AT(delp + o, i, j) * ar;
            double x = which == 0 ? m : (which == 1 ? (double)AT(pt + o, i, j) * m : (double)AT(q + o, i, j) * m);
            neu_add(s, c, x);
        }
    }
    ss[tid] = s;
    sc[tid] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            double a = ss[tid], ac = sc[tid] + sc[tid + w];
            neu_add(a, ac, ss[tid + w]);
            ss[tid] = a;
            sc[tid] = ac;
        }
        __syncthreads();
    }
    if (tid == 0) {
        long b = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[2 * b] = ss[0];
        part[2 * b + 1] = sc[0];
    }
}

// ====================================================================
// Workspace carve-up
// ====================================================================
struct Work {
    // bulk layer fields
    B *ua, *va, *ucp, *vcp, *ax, *ay, *Fm, *Fp, *Fw, *Gm, *Gp, *Gw, *delpc, *ptc, *wc, *ke, *vort;
    B *ut, *vt, *crx, *cry, *xfx, *yfx, *FX, *FY, *GX, *GY, *WX, *WY, *dn, *pn, *wn, *om, *VX, *VY;
    B *cxI, *cyI, *xI, *yI, *tfx2, *tfy2, *tqi, *tqj;
    // FP64 fields
    double *pkc, *gz, *delzc, *zh, *zn, *ZX, *ZY, *s1, *s2, *s3, *pB, *zB, *dB;
    double *zfx2, *zfy2, *zqi, *zqj, *dp1, *dp2, *mxs, *mys;
    unsigned long long *umax;
    double *part;
};

long reduction_elems(const fv3_grid *g);
static long part_count(const fv3_grid *g)
{
    long bx = (g->n + 63) / 64, by = (g->n + 3) / 4;
    return bx * by * g->T;
}

static size_t carve(const fv3_grid *g, char *base, Work *w)
{
    long el = alloc_elems(g, g->nz), ei = alloc_elems(g, g->nz + 1);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    B **bulk[] = {&w->ua, &w->va, &w->ucp, &w->vcp, &w->ax, &w->ay, &w->Fm, &w->Fp, &w->Fw, &w->Gm,
                  &w->Gp, &w->Gw, &w->delpc, &w->ptc, &w->wc, &w->ke, &w->vort, &w->ut, &w->vt,
                  &w->crx, &w->cry, &w->xfx, &w->yfx, &w->FX, &w->FY, &w->GX, &w->GY, &w->WX,
                  &w->WY, &w->dn, &w->pn, &w->wn, &w->om, &w->VX, &w->VY, &w->cxI, &w->cyI,
                  &w->xI, &w->yI, &w->tfx2, &w->tfy2, &w->tqi, &w->tqj};
    for (auto p : bulk) *p = (B *)take(el * sizeof(B));
    double **f64[] = {&w->delzc, &w->ZX, &w->ZY, &w->s1, &w->s2, &w->s3, &w->dB, &w->zfx2,
                      &w->zfy2, &w->zqi, &w->zqj, &w->dp1, &w->dp2, &w->mxs, &w->mys};
    for (auto p : f64) *p = (double *)take(el * sizeof(double));
    double **f64i[] = {&w->pkc, &w->gz, &w->zh, &w->zn, &w->pB, &w->zB};
    for (auto p : f64i) *p = (double *)take(ei * sizeof(double));
    w->umax = (unsigned long long *)take(64);
    w->part = (double *)take(2 * part_count(g) * sizeof(double));
    return off + 256;
}

long reduction_elems(const fv3_grid *g) { return 2 * part_count(g); }

void timing_start(const char *filter)
{
    g_timing.on = filter != nullptr;
    g_timing.filter = filter ? filter : "";
    g_timing.recs.clear();
}

int timing_stop(char *names, int names_cap, double *total_ms, long *counts, int cap)
{
    g_timing.on = false;
    if (hipDeviceSynchronize() != hipSuccess) return (int)FV3_EDEVICE;
    std::vector<std::string> keys;
    std::vector<double> tot;
    std::vector<long> cnt;
    for (TimingRec &r : g_timing.recs) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        size_t q = 0;
        while (q < keys.size() && keys[q] != r.name) q++;
        if (q == keys.size()) {
            keys.push_back(r.name);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[q] += ms;
        cnt[q] += 1;
    }
    g_timing.recs.clear();
    int nk = 0, pos = 0;
    for (size_t q = 0; q < keys.size() && nk < cap; q++) {
        int len = (int)keys[q].size() + 1;
        if (pos + len > names_cap) break;
        std::memcpy(names + pos, keys[q].c_str(), len);
        pos += len;
        total_ms[nk] = tot[q];
        counts[nk] = cnt[q];
        nk++;
    }
    return nk;
}

size_t workspace_bytes(const fv3_grid *g)
{
    Work w;
    return carve(g, nullptr, &w);
}

static Met metrics(const fv3_grid *g)
{
    Met M;
    for (int m = 0; m < M_COUNT; m++) M.m[m] = g->met[m];
    return M;
}

// ====================================================================
// Host orchestration of one call
// ====================================================================
fv3_status run_substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split, int stop_stage,
                        hipStream_t st)
{
    if (g->bulk_bytes != (int)sizeof(B)) return FV3_EUNSUPPORTED;
    Work W;
    carve(g, (char *)s->workspace, &W);
    Met M = metrics(g);
    const Geo &G = g->geo;
    int n = g->n, nz = g->nz, T = g->T, P = T * nz;
    long el = alloc_elems(g, nz);
    B *u = (B *)s->u, *v = (B *)s->v, *w = (B *)s->w, *delp = (B *)s->delp, *pt = (B *)s->pt;
    B *uc = (B *)s->uc, *vc = (B *)s->vc, *cx = (B *)s->cx, *cy = (B *)s->cy;
    double *delz = s->delz;
    const double *phis = s->phis;
    double bdt = dt / n_split, dt2 = 0.5 * bdt;

    fill(s->mfx, el, 0.0, st);
    fill(s->mfy, el, 0.0, st);
    fill(cx, el, (B)0, st);
    fill(cy, el, (B)0, st);
    copy(delp, s->dp0, el, st);
    FvTmp tb{W.tfx2, W.tfy2, W.tqi, W.tqj};
    FvTmp tz{W.zfx2, W.zfy2, W.zqi, W.zqj};

    for (int it = 0; it < n_split; it++) {
        bool last = it == n_split - 1;
#define STOP(x) if (last && stop_stage == (x)) goto done
        // H-A
        halo_pair(g, g->planD, u, v, nz, st);
        halo_scalar(g, delp, nz, st);
        halo_scalar(g, pt, nz, st);
        halo_scalar(g, w, nz, st);
        halo_scalar(g, delz, nz, st);
        STOP(1);
        // c_sw
        launch2d(k_csw_agrid, -3, n + 2, -3, n + 2, P, st, G, (const B *)u, (const B *)v, W.ua, W.va);
        launch2d(k_csw_faces, -1, n + 1, -1, n + 1, P, st, G, M, (B)dt2, (const B *)u, (const B *)v,
                 (const B *)delp, (const B *)pt, (const B *)w, (const B *)W.ua, (const B *)W.va, W.ucp, W.vcp,
                 W.ax, W.ay, W.Fm, W.Fp, W.Fw, W.Gm, W.Gp, W.Gw);
        launch2d(k_csw_cells, -1, n, -1, n, P, st, G, M, (B)dt2, (const B *)delp, (const B *)pt, (const B *)w,
                 (const B *)W.ua, (const B *)W.va, (const B *)W.ucp, (const B *)W.vcp, (const B *)W.Fm,
                 (const B *)W.Fp, (const B *)W.Fw, (const B *)W.Gm, (const B *)W.Gp, (const B *)W.Gw, W.delpc,
                 W.ptc, W.wc, W.ke, W.vort);
        launch2d(k_csw_update, 0, n, 0, n, P, st, G, M, (B)dt2, (const B *)u, (const B *)v, (const B *)W.ucp,
                 (const B *)W.vcp, (const B *)W.ke, (const B *)W.vort, uc, vc);
        STOP(2);
        // dz_c + riem_solver_c on the half-step cells
        launch2d(k_dzc, -1, n, -1, n, T, st, G, M, (const double *)delz, phis, (const B *)W.ax, (const B *)W.ay,
                 W.delzc);
        launch2d(k_sim1<B>, -1, n, -1, n, T, st, G, dt2, g->p.ptop, (const B *)W.delpc, (const B *)W.ptc,
                 (const double *)W.delzc, (const B *)W.wc, phis, W.s1, W.s2, W.s3, (B *)nullptr,
                 (double *)nullptr, W.pkc, W.gz, 1);
        STOP(3);
        launch2d(k_pgradc, 0, n, 0, n, P, st, G, M, dt2, (const B *)W.delpc, (const double *)W.pkc,
                 (const double *)W.gz, uc, vc);
        STOP(4);
        halo_pair(g, g->planCv, uc, vc, nz, st);
        STOP(5);
        // d_sw
        launch2d(k_dsw_courant, -3, n + 2, -3, n + 2, P, st, G, M, (B)bdt, (const B *)uc, (const B *)vc, W.ut,
                 W.vt, W.crx, W.cry, W.xfx, W.yfx, g->flags);
        fv_tp_2d<B, B>(g, M, nz, nz, P, delp, W.crx, W.cry, W.xfx, W.yfx, (const B *)nullptr,
                       (const B *)nullptr, W.FX, W.FY, tb, st);
        launch2d(k_dsw_mass, 0, n, 0, n, P, st, G, M, (const B *)delp, (const B *)W.FX, (const B *)W.FY,
                 (const B *)W.crx, (const B *)W.cry, W.dn, s->mfx, s->mfy, cx, cy);
        fv_tp_2d<B, B>(g, M, nz, nz, P, pt, W.crx, W.cry, W.xfx, W.yfx, (const B *)W.FX, (const B *)W.FY, W.GX,
                       W.GY, tb, st);
        launch2d(k_dsw_scalar, 0, n - 1, 0, n - 1, P, st, G, M, (const B *)pt, (const B *)delp, (const B *)W.dn,
                 (const B *)W.GX, (const B *)W.GY, W.pn);
        fv_tp_2d<B, B>(g, M, nz, nz, P, w, W.crx, W.cry, W.xfx, W.yfx, (const B *)W.FX, (const B *)W.FY, W.WX,
                       W.WY, tb, st);
        launch2d(k_dsw_scalar, 0, n - 1, 0, n - 1, P, st, G, M, (const B *)w, (const B *)delp, (const B *)W.dn,
                 (const B *)W.WX, (const B *)W.WY, W.wn);
        launch2d(k_dsw_ke, 0, n, 0, n, P, st, G, M, (B)bdt, (const B *)u, (const B *)v, (const B *)W.ut,
                 (const B *)W.vt, W.ke);
        launch2d(k_dsw_omega, -3, n + 2, -3, n + 2, P, st, G, M, (const B *)u, (const B *)v, W.om);
        fv_tp_2d<B, B>(g, M, nz, nz, P, W.om, W.crx, W.cry, W.xfx, W.yfx, (const B *)nullptr, (const B *)nullptr,
                       W.VX, W.VY, tb, st);
        launch2d(k_dsw_update, 0, n, 0, n, P, st, G, M, (const B *)W.ke, (const B *)W.VX, (const B *)W.VY,
                 (const B *)W.dn, (const B *)W.pn, (const B *)W.wn, u, v, delp, pt, w);
        STOP(6);
        // dz_d
        launch2d(k_heights, -3, n + 2, -3, n + 2, T, st, G, (const double *)delz, phis, W.zh);
        launch2d(k_iface_flux, -3, n + 3, -3, n + 3, P, st, G, (const B *)W.crx, (const B *)W.cry,
                 (const B *)W.xfx, (const B *)W.yfx, W.cxI, W.cyI, W.xI, W.yI);
        fv_tp_2d<double, double>(g, M, nz + 1, nz, P, W.zh, W.cxI, W.cyI, W.xI, W.yI, (const double *)nullptr,
                                 (const double *)nullptr, W.ZX, W.ZY, tz, st);
        launch2d(k_zh_update, 0, n - 1, 0, n - 1, P, st, G, M, (const double *)W.zh, (const double *)W.ZX,
                 (const double *)W.ZY, (const B *)W.xI, (const B *)W.yI, W.zn);
        launch2d(k_delz_from_zh, 0, n - 1, 0, n - 1, P, st, G, (const double *)W.zn, phis, delz);
        STOP(7);
        // riem_solver3
        launch2d(k_sim1<B>, 0, n - 1, 0, n - 1, T, st, G, bdt, g->p.ptop, (const B *)delp, (const B *)pt,
                 (const double *)delz, (const B *)w, phis, W.s1, W.s2, W.s3, w, delz, s->pfull, s->phi, 0);
        STOP(8);
        // H-C
        halo_scalar(g, s->pfull, nz + 1, st);
        halo_scalar(g, s->phi, nz + 1, st);
        halo_scalar(g, delp, nz, st);
        STOP(9);
        // nh_p_grad
        launch2d(k_corner_interp<double>, 0, n, 0, n, T * (nz + 1), st, G, nz + 1, (const double *)s->pfull, W.pB);
        launch2d(k_corner_interp<double>, 0, n, 0, n, T * (nz + 1), st, G, nz + 1, (const double *)s->phi, W.zB);
        launch2d(k_corner_interp<B>, 0, n, 0, n, P, st, G, nz, (const B *)delp, W.dB);
        launch2d(k_nhpgrad, 0, n, 0, n, P, st, G, M, bdt, (const double *)W.pB, (const double *)W.zB,
                 (const double *)W.dB, u, v);
#undef STOP
    }
done:
    {
        B *chk[] = {u, v, w, delp, pt};
        for (B *f : chk) launch2d(k_check_finite<B>, 0, n - 1, 0, n - 1, P, st, G, nz, (const B *)f, g->flags);
        launch2d(k_check_finite<double>, 0, n - 1, 0, n - 1, P, st, G, nz, (const double *)delz, g->flags);
    }
    if (hipGetLastError() != hipSuccess) return FV3_EDEVICE;
    return FV3_OK;
}

fv3_status run_halo_cells(const fv3_grid *g, void *const *f, int nf, int levels, int fp64,
                          hipStream_t st)
{
    for (int q = 0; q < nf; q++) {
        if (fp64 || sizeof(B) == 8) halo_scalar(g, (double *)f[q], levels, st);
    }
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

fv3_status run_tracer(void *const *q, int nq, fv3_state *s, const fv3_grid *g, int nsplt,
                      hipStream_t st)
{
    if (g->bulk_bytes != (int)sizeof(B)) return FV3_EUNSUPPORTED;
    Work W;
    carve(g, (char *)s->workspace, &W);
    Met M = metrics(g);
    const Geo &G = g->geo;
    int n = g->n, nz = g->nz, T = g->T, P = T * nz;
    long el = alloc_elems(g, nz);
    B *cx = (B *)s->cx, *cy = (B *)s->cy;
    halo_pair(g, g->planCv, cx, cy, nz, st);
    if (nsplt <= 0) {
        unsigned long long zero = 0, h = 0;
        fill(W.umax, 1, zero, st);
        launch2d(k_absmax, 0, n, 0, n, P, st, G, (const B *)cx, (const B *)cy, W.umax);
        if (hipMemcpyAsync(&h, W.umax, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return FV3_EDEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return FV3_EDEVICE;
        double cmax;
        std::memcpy(&cmax, &h, sizeof(cmax));
        nsplt = (int)std::ceil(cmax);
        if (nsplt < 1) nsplt = 1;
    }
    double rs = (double)nsplt;
    launch2d(k_tracer_flux, -3, n + 3, -3, n + 3, P, st, G, M, rs, (const B *)cx, (const B *)cy,
             (const double *)s->mfx, (const double *)s->mfy, W.crx, W.cry, W.xfx, W.yfx, W.mxs, W.mys);
    copy(s->dp0, W.dp1, el, st);
    double *dp1 = W.dp1, *dp2 = W.dp2;
    FvTmp tb{W.tfx2, W.tfy2, W.tqi, W.tqj};
    for (int itr = 0; itr < nsplt; itr++) {
        launch2d(k_tracer_dp, 0, n - 1, 0, n - 1, P, st, G, M, (const double *)dp1, (const double *)W.mxs,
                 (const double *)W.mys, dp2);
        for (int m = 0; m < nq; m++) {
            B *Q = (B *)q[m];
            halo_scalar(g, Q, nz, st);
            fv_tp_2d<B, double>(g, M, nz, nz, P, Q, W.crx, W.cry, W.xfx, W.yfx, (const double *)W.mxs,
                                (const double *)W.mys, W.FX, W.FY, tb, st);
            launch2d(k_tracer_update, 0, n - 1, 0, n - 1, P, st, G, M, (const double *)dp1, (const double *)dp2,
                     (const B *)W.FX, (const B *)W.FY, Q);
        }
        double *tmp = dp1;
        dp1 = dp2;
        dp2 = tmp;
    }
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

fv3_status run_mass_sums(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                         int nq, double *out, hipStream_t st)
{
    if (g->bulk_bytes != (int)sizeof(B)) return FV3_EUNSUPPORTED;
    Met M = metrics(g);
    const Geo &G = g->geo;
    int n = g->n;
    long np = part_count(g);
    double *part = g->red;
    std::vector<double> h(2 * np);
    for (int which = 0; which < 2 + nq; which++) {
        const B *qq = which >= 2 ? (const B *)q[which - 2] : nullptr;
        launch2d(k_mass_partial, 0, n - 1, 0, n - 1, g->T, st, G, M, (const B *)delp, (const B *)pt, qq,
                 which < 2 ? which : 2, part);
        if (hipMemcpyAsync(h.data(), part, 2 * np * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
            return FV3_EDEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return FV3_EDEVICE;
        double s = 0.0, c = 0.0;
        for (long b = 0; b < np; b++) {
            c += h[2 * b + 1];
            double x = h[2 * b], t = s + x;
            if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
            else c += (x - t) + s;
            s = t;
        }
        out[which] = s + c;
    }
    return FV3_OK;
}

}  // namespace fv3
