// HIP kernels of the FV3 acoustic substep loop and tracer transport (gfx950).
//
// Data layout: every field is [tile][level][row][column], column index i
// contiguous (coalesced across the 64 lanes of a wavefront), halo of 3 points,
// rows padded to 128 bytes with interior i = 0 aligned.  Kernels are
// templated on the bulk type B (double, or float for the mixed-precision
// build); the column solves, vertical scans, pressure gradients and mass-flux
// accumulators are always FP64.
//
// Stencil kernels work on one (tile, level) plane per grid z index.  The
// flux-form transport fv_tp_2d (paper Sec. IX-C) is one fused kernel: a
// 64 x 16 cell tile with its 3-point halo is staged in LDS, and the outer
// fluxes, inner advective updates, final fluxes and the flux-divergence update
// of the transported field all run out of LDS.  Corner blocks of cube tiles
// are never stored: reads of them are remapped to the adjacent edge halo
// rotated about the cube vertex, in the x-sweep or y-sweep sense of the
// reading stencil (generalising the corner statement of Sec. VII-C).  Column
// kernels march k in one thread per column with software-pipelined loads.
//
// The order of the stages inside a substep follows the FV3 acoustic loop
// (Sec. II): halo A, c_sw, dz_c + riem_solver_c, p_grad_c, halo B, d_sw,
// dz_d + riem_solver3, halo C, nh_p_grad.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <utility>
#include <string>
#include <vector>

#include "fv3_internal.hpp"
#include "flog.hpp"

namespace fv3 {

#define DEVI __device__ __forceinline__

// ------------------------------------------------------------ indexing
DEVI long pidx(const Geo &G, int L, int t, int k) { return G.off0 + ((long)t * L + k) * G.lev; }
// Element (i, j) of a plane whose interior origin is P (i, j >= -3): the
// address is the plane's halo corner (-3, -3) plus a non-negative 32-bit
// byte offset, so that a block-uniform P becomes a scalar base with one
// 32-bit vector offset instead of per-lane 64-bit address arithmetic.
template <class T>
DEVI T &at_(T *p, int i, int j, int pitch)
{
    char *b = (char *)(p - (3 * pitch + 3));
    return *(T *)(b + (unsigned)((j + 3) * pitch + (i + 3)) * (unsigned)sizeof(T));
}
#define AT(P, i, j) at_((P), (int)(i), (int)(j), (int)G.pitch)

// a / b in the FP32 bulk through the hardware reciprocal (about 1 ulp, far
// below the FP32 bulk's rounding), FP64 exact
template <class T>
DEVI T rdiv(T a, T b)
{
    if constexpr (std::is_same<T, float>::value) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

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
    int i = ib + (int)(bk.x * blockDim.x + threadIdx.x);       \
    int j = jlo + (int)(bk.y * blockDim.y + threadIdx.y);      \
    if (i < ilo || i > ihi || j > jhi) return;                       \
    int t = (int)bk.z / (L), k = (int)bk.z % (L);        \
    (void)t; (void)k;

// Plane kernels: point range [ilo, ihi] x [jlo, jhi]; thread columns start at
// ib <= ilo, a multiple of 32 elements from the interior origin, so that every
// wavefront's 64 columns begin on a 128-byte line (interior column 0 is
// line-aligned in the layout).
#define KARGS Bk bk, int ib, int ilo, int ihi, int jlo, int jhi

template <class R>
struct Mets {
    const R *m[M_ALL];
};
typedef Mets<double> MetD;

// plane pointer of a 2-D metric for tile t
#define MP(M, name) ((M).m[name] + G.off0 + (long)t * G.lev)

// ---------------------------------------------------------- launch timing
static struct {
    bool on = false;
    std::string filter;
    std::vector<TimingRec> recs;
} g_timing;

bool timing_wanted(const char *name)
{
    return g_timing.on && std::strstr(name, g_timing.filter.c_str()) != nullptr;
}
void timing_begin(const char *name, hipStream_t st, TimingRec &r)
{
    r.name = name;
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, st);
}
void timing_end(hipStream_t st, TimingRec &r)
{
    (void)hipEventRecord(r.b, st);
    g_timing.recs.push_back(r);
}

// ---------------------------------------------------------- kernel launch
// Every kernel of the substep path is a device function that takes its block
// index explicitly.  It is launched either alone (k_one: the block index is
// the hardware one), or for an ensemble of grids in one launch (k_multi: grid
// z runs over the planes of all members, each block looks its member up in a
// small table and reads that member's arguments from device memory; blocks
// outside the member's own x/y extent exit at once).  Both paths run the same
// device code, so an ensemble member computes exactly what it computes alone.
template <class... A>
struct Tup;
template <>
struct Tup<> {
};
template <class H, class... R>
struct Tup<H, R...> {
    H h;
    Tup<R...> r;
};
static inline Tup<> tup() { return {}; }
template <class H, class... R>
static Tup<H, R...> tup(H h, R... r)
{
    return Tup<H, R...>{h, tup(r...)};
}
template <size_t I, class H, class... R>
DEVI const auto &tget(const Tup<H, R...> &t)
{
    if constexpr (I == 0) return t.h;
    else return tget<I - 1>(t.r);
}
template <auto F, class... A, size_t... I>
DEVI void tcall(Bk bk, const Tup<A...> &t, std::index_sequence<I...>)
{
    F(bk, tget<I>(t)...);
}

// MI355X hands consecutive workgroups of a launch to its eight XCDs in turn,
// and each XCD has its own L2.  The block index a kernel body sees is
// therefore permuted so that every XCD works on one contiguous range of the
// grid (x fastest, then y, then z): neighbouring tiles, which share halo
// lines, and the planes of one tile, which share the 2-D metric terms, then
// meet in the same L2.  The permutation is a bijection of the grid.
constexpr unsigned NXCD = 8;
DEVI Bk xcd_block()
{
    const unsigned gx = gridDim.x, gy = gridDim.y, total = gx * gy * gridDim.z;
    const unsigned id = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned q = total / NXCD, rem = total % NXCD, xcd = id % NXCD, local = id / NXCD;
    const unsigned lid = xcd * q + (xcd < rem ? xcd : rem) + local;
    return Bk{lid % gx, (lid / gx) % gy, lid / (gx * gy)};
}

// Minimum wavefronts per SIMD a kernel body is compiled for (its register
// budget: at most 512 / waves VGPRs); 1 leaves the choice to the compiler.
template <auto F>
constexpr int kocc = 1;

template <auto F, class... A>
__global__ void __launch_bounds__(256, kocc<F>) k_one(A... a)
{
    F(xcd_block(), a...);
}

template <auto F, class... A>
__global__ void __launch_bounds__(256, kocc<F>) k_multi(const Tup<A...> *__restrict__ args, const MemberBlk *__restrict__ tab,
                                               int members)
{
    // one-dimensional grid over every member's own blocks back to back (no
    // block outside a member's extent): find the member, then its block
    const int L = (int)xcd_block().x;
    int lo = 0, hi = members - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tab[mid].b0 <= L) lo = mid;
        else hi = mid - 1;
    }
    const MemberBlk mb = tab[lo];
    const int gxy = mb.gx * mb.gy, local = L - mb.b0;
    if (gxy <= 0) return;
    const int bz = local / gxy, rem = local - bz * gxy, by = rem / mb.gx, bx = rem - by * mb.gx;
    if (bz >= mb.gz) return;
    tcall<F>(Bk{(unsigned)bx, (unsigned)by, (unsigned)bz}, args[lo], std::index_sequence_for<A...>{});
}

// Recording of the launch sequence of one call per member (ensemble mode).
static thread_local Recorder *g_rec = nullptr;

template <class Tp>
static void rec_site(const char *name, const void *km, bool tunable, dim3 blk, int ex, int ey, int ez, const Tp &t)
{
    Recorder &R = *g_rec;
    if (R.member == 0) {
        Site s;
        s.name = name;
        s.kmulti = km;
        s.argsz = sizeof(Tp);
        s.tunable = tunable;
        s.blk = blk;
        R.sites.push_back(std::move(s));
    }
    if (R.pos >= R.sites.size() || R.sites[R.pos].kmulti != km) {
        R.bad = true;
        return;
    }
    Site &s = R.sites[R.pos++];
    const char *b = (const char *)&t;
    s.blob.insert(s.blob.end(), b, b + sizeof(Tp));
    s.ex.push_back(ex);
    s.ey.push_back(ey);
    s.ez.push_back(ez);
}

// marks the boundaries entry | substep | exit of the recorded sequence
static void rec_mark()
{
    if (!g_rec) return;
    Recorder &R = *g_rec;
    if (R.member == 0) R.marks.push_back(R.pos);
    else if (R.mark >= R.marks.size() || R.marks[R.mark] != R.pos) R.bad = true;
    R.mark++;
}

// plane kernels: 64 x 4 threads, one point each, grid z = planes
// Block shape of a plane kernel: 256 threads, bx consecutive points along i
// (a multiple of 16, so that a wavefront's row segments are whole 64-byte
// lines for FP32 and 128-byte lines for FP64).
struct Shape {
    int x, y;
};
constexpr Shape SH_DEFAULT{64, 4};

template <auto F, class... A>
static void launch2d_sh(const char *name, Shape sh, int ilo, int ihi, int jlo, int jhi, int planes,
                        hipStream_t st, A... a)
{
    // columns start at an aligned point: ilo itself, or -min(bx, 32) for halo ranges
    const int ib = ilo >= 0 ? ilo : -(sh.x < 32 ? sh.x : 32);
    if (g_rec) {
        rec_site(name, (const void *)k_multi<F, int, int, int, int, int, A...>, true, dim3(sh.x, sh.y, 1),
                 ihi - ib + 1, jhi - jlo + 1, planes, tup(ib, ilo, ihi, jlo, jhi, a...));
        return;
    }
    dim3 blk((unsigned)sh.x, (unsigned)sh.y, 1);
    dim3 grd((unsigned)((ihi - ib + sh.x) / sh.x), (unsigned)((jhi - jlo + sh.y) / sh.y), (unsigned)planes);
    bool tm = timing_wanted(name);
    TimingRec r;
    if (tm) timing_begin(name, st, r);
    hipLaunchKernelGGL((k_one<F, int, int, int, int, int, A...>), grd, blk, 0, st, ib, ilo, ihi, jlo, jhi, a...);
    if (tm) timing_end(st, r);
}
template <auto F, class... A>
static void launch2d_fn(const char *name, int ilo, int ihi, int jlo, int jhi, int planes, hipStream_t st, A... a)
{
    launch2d_sh<F>(name, SH_DEFAULT, ilo, ihi, jlo, jhi, planes, st, a...);
}
#define launch2d(kern, ...) launch2d_fn<kern>(#kern, __VA_ARGS__)
// with a block shape chosen per kernel (measured on MI355X at C192 x 79)
#define launch2d_s(kern, shape, ...) launch2d_sh<kern>(#kern, shape, __VA_ARGS__)

// generic launch with explicit shape (timed under `name`)
template <auto F, class... A>
static void launch_fn(const char *name, dim3 grd, dim3 blk, hipStream_t st, A... a)
{
    if (g_rec) {
        rec_site(name, (const void *)k_multi<F, A...>, false, blk, (int)grd.x, (int)grd.y, (int)grd.z, tup(a...));
        return;
    }
    bool tm = timing_wanted(name);
    TimingRec r;
    if (tm) timing_begin(name, st, r);
    hipLaunchKernelGGL((k_one<F, A...>), grd, blk, 0, st, a...);
    if (tm) timing_end(st, r);
}

// plain __global__ kernels outside the substep path (reductions)
template <class Kern, class... A>
static void launch2d_native(const char *name, Kern kern, int ilo, int ihi, int jlo, int jhi, int planes,
                            hipStream_t st, A... a)
{
    dim3 blk(64, 4, 1);
    dim3 grd((unsigned)((ihi - ilo + 64) / 64), (unsigned)((jhi - jlo + 4) / 4), (unsigned)planes);
    bool tm = timing_wanted(name);
    TimingRec r;
    if (tm) timing_begin(name, st, r);
    hipLaunchKernelGGL(kern, grd, blk, 0, st, ilo, ihi, jlo, jhi, a...);
    if (tm) timing_end(st, r);
}

// ====================================================================
// 1-D PPM face value: face between cells m-1 and m along a sweep, cell
// values q0..q5 = cells m-3..m+2, Courant number c, order ORD.
//  8 monotone: limited slope per cell (zero at extrema), fourth-order edge
//    values, edge deviations clipped to twice the slope with the slope's
//    sign, mean of the parabola over the swept part of the upwind cell;
//  6 unlimited: slopes (q+ - q-)/4 and the edge deviations as they come;
//  5 2dx-filtered: order 6, but the upwind cell mean where that cell and a
//    neighbour are both strict local extrema (an oscillation over 2 cells);
//  7 positive-definite (tracers): order 6 with the parabola of a cell of
//    non-negative mean q scaled about q by q / (q - min) where its minimum
//    over the cell is negative (Zhang & Shu's scaling limiter).
// ====================================================================
template <class T>
DEVI T lslope(T a, T b, T c)
{
    // zero at an extremum of (a, b, c): then min(mx - b, b - mn) is zero
    T d = (c - a) * (T)0.25;
    T mx = fmax(a, fmax(b, c)), mn = fmin(a, fmin(b, c));
    return copysign(fmin(fabs(d), fmin(mx - b, b - mn)), d);
}

// Face value from the upwind cell q's parabola (neighbours a, b | d, e), with
// c the signed Courant number.  For the downwind orientation the parabola's
// edge deviations swap roles and the swept fraction is |c|:
// q + (1 - |c|) (e - |c| (bl + br)), e = br for c > 0 and bl otherwise.
template <int ORD, class T>
DEVI T ppm_up(T a, T b, T q, T d, T e, T c)
{
    const T third = (T)1 / (T)3;
    if constexpr (ORD == 5) {
        const bool xb = (b - a) * (q - b) < (T)0, xq = (q - b) * (d - q) < (T)0, xd = (d - q) * (e - d) < (T)0;
        if (xq && (xb || xd)) return q;
    }
    T bl, br;
    if constexpr (ORD == 8) {
        const T dl = lslope(a, b, q), dm = lslope(b, q, d), dr = lslope(q, d, e);
        const T al = (T)0.5 * (b + q) + (dl - dm) * third;
        const T ar = (T)0.5 * (q + d) + (dm - dr) * third;
        // deviations clipped to twice the slope, with the slope's sign (zero slope: zero)
        const T a2 = (T)2 * fabs(dm);
        bl = copysign(fmin(a2, fabs(al - q)), -dm);
        br = copysign(fmin(a2, fabs(ar - q)), dm);
    } else {
        const T qt = (T)0.25;
        const T dl = (q - a) * qt, dm = (d - b) * qt, dr = (e - q) * qt;
        bl = (T)0.5 * (b + q) + (dl - dm) * third - q;
        br = (T)0.5 * (q + d) + (dm - dr) * third - q;
    }
    if constexpr (ORD == 7) {
        if (q >= (T)0) {
            // minimum over the cell: an edge, or the vertex when it is a
            // minimum (a6 < 0) inside the cell (|aR - aL| < -a6)
            const T aL = q + bl, aR = q + br, a6 = (T)-3 * (bl + br), da = aR - aL;
            T mn = fmin(aL, aR);
            if (a6 < (T)0 && fabs(da) < -a6) mn = fmin(mn, q + da * da / ((T)4 * a6) + a6 / (T)12);
            if (mn < (T)0) {
                const T th = q / (q - mn);
                bl *= th;
                br *= th;
            }
        }
    }
    const T cc = fabs(c);
    return q + ((T)1 - cc) * ((c > 0 ? br : bl) - cc * (bl + br));
}

template <int ORD, class T>
DEVI T ppm6(T q0, T q1, T q2, T q3, T q4, T q5, T c)
{
    // Branch-free: select the upwind cell's five-point neighbourhood (cell
    // m-1 for c > 0, else cell m), then one evaluation.
    const bool pos = c > 0;
    return ppm_up<ORD>(pos ? q0 : q1, pos ? q1 : q2, pos ? q2 : q3, pos ? q3 : q4, pos ? q4 : q5, c);
}

// The same from six cells m-3..m+2 stored S apart from p (in LDS): the upwind
// neighbourhood is selected by its address, five loads instead of six.
template <int S, int ORD, class T>
DEVI T ppm_lds(const T *p, T c)
{
    const T *u = p + (c > 0 ? 0 : S);
    return ppm_up<ORD>(u[0], u[S], u[2 * S], u[3 * S], u[4 * S], c);
}

// Face value next to a cube tile edge (option edge_ppm, Putman & Lin 2007).
// p holds the six cells m-3..m+2 of the sweep, S apart; w their widths along
// the sweep, ws apart.  Window interface pe (between window cells pe-1 and
// pe, 1 <= pe <= 5) is the edge; the tile lies at cells >= pe (west) or
// below pe.  The edge values of the three interfaces around the edge are
// one-sided: at the edge, the mean of the linear extrapolations from the two
// cells on either side (by distance); next to it, three cells of its own
// side, (3 q_near + 11 q_far) / 14 -+ (4/7) times the far cell's slope.
// Order 8 leaves the deviations of the two cells beside the edge and of the
// second cell inside the tile unclipped and makes their parabolas monotone
// (Colella & Woodward 1984).  Written without dynamically indexed arrays.
template <int ORD, class T>
DEVI T ppm_edge(const T *p, int S, const T *w, int ws, T c, int pe, bool west)
{
    T q[6], x[6], dm[6], al[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        q[k] = p[k * S];
        x[k] = w[k * ws];
    }
    const bool pos = c > 0;
    if constexpr (ORD == 5) {
        const bool x1 = (q[1] - q[0]) * (q[2] - q[1]) < (T)0, x2 = (q[2] - q[1]) * (q[3] - q[2]) < (T)0;
        const bool x3 = (q[3] - q[2]) * (q[4] - q[3]) < (T)0, x4 = (q[4] - q[3]) * (q[5] - q[4]) < (T)0;
        if (pos ? (x2 && (x1 || x3)) : (x3 && (x2 || x4))) return pos ? q[2] : q[3];
    }
#pragma unroll
    for (int k = 1; k <= 4; k++)
        dm[k] = ORD == 8 ? lslope(q[k - 1], q[k], q[k + 1]) : (q[k + 1] - q[k - 1]) * (T)0.25;
    const T third = (T)1 / (T)3, r14 = (T)1 / (T)14, f47 = (T)4 / (T)7;
#pragma unroll
    for (int k = 2; k <= 4; k++) {
        T v = (T)0.5 * (q[k - 1] + q[k]) + (dm[k - 1] - dm[k]) * third;
        if (k == pe) {
            const T lo = (((T)2 * x[k - 1] + x[k - 2]) * q[k - 1] - x[k - 1] * q[k - 2]) / (x[k - 2] + x[k - 1]);
            const T hi = (((T)2 * x[k] + x[k + 1]) * q[k] - x[k] * q[k + 1]) / (x[k] + x[k + 1]);
            v = (T)0.5 * (lo + hi);
        } else if (k == pe - 1) {
            v = ((T)3 * q[k] + (T)11 * q[k - 1]) * r14 + f47 * dm[k - 1];
        } else if (k == pe + 1) {
            v = ((T)3 * q[k - 1] + (T)11 * q[k]) * r14 - f47 * dm[k];
        }
        al[k] = v;
    }
    const int s = pos ? 2 : 3;
    const T qs = pos ? q[2] : q[3], ds = pos ? dm[2] : dm[3];
    const T aL = pos ? al[2] : al[3], aR = pos ? al[3] : al[4];
    const bool edge_cell = s == pe - 1 || s == pe || s == (west ? pe + 1 : pe - 2);
    T bl = aL - qs, br = aR - qs;
    if constexpr (ORD == 8) {
        if (!edge_cell) {
            const T a2 = (T)2 * fabs(ds);
            bl = copysign(fmin(a2, fabs(bl)), -ds);
            br = copysign(fmin(a2, fabs(br)), ds);
        } else if (bl * br >= (T)0) {
            bl = br = (T)0;
        } else {
            const T da = br - bl, a6 = (T)-3 * (bl + br);
            if (a6 * da > da * da) bl = (T)-2 * br;
            else if (a6 * da < -(da * da)) br = (T)-2 * bl;
        }
    }
    if constexpr (ORD == 7) {
        if (qs >= (T)0) {
            const T eL = qs + bl, eR = qs + br, a6 = (T)-3 * (bl + br), da = eR - eL;
            T mn = fmin(eL, eR);
            if (a6 < (T)0 && fabs(da) < -a6) mn = fmin(mn, qs + da * da / ((T)4 * a6) + a6 / (T)12);
            if (mn < (T)0) {
                const T th = qs / (qs - mn);
                bl *= th;
                br *= th;
            }
        }
    }
    const T cc = fabs(c);
    return qs + ((T)1 - cc) * ((pos ? br : bl) - cc * (bl + br));
}

// Window position of a tile edge for face m of a sweep over n cells, or 0
// when the face has no edge cell upwind (faces 0, 1, 2 and n-2, n-1, n do).
DEVI int edge_pe(int m, int n, bool &west)
{
    west = m <= 2;
    if (m >= 0 && m <= 2) return 3 - m;
    if (m >= n - 2 && m <= n) return n - m + 3;
    return 0;
}
DEVI bool edge_face(int m, int n) { return m <= 2 || m >= n - 2; }
// the k-th (0..5) face with an edge cell upwind: 0, 1, 2, n-2, n-1, n
DEVI int edge_face_at(int k, int n) { return k < 3 ? k : n - 5 + k; }

// ====================================================================
// Halo exchange: plan-driven copies from the neighbour tile's interior
// (orientation transform folded into the plan for vector pairs).
// ====================================================================
template <class T>
DEVI void k_halo_scalar(Bk bk, Geo G, const HaloEnt *__restrict__ plan, int count, T *f, int L)
{
    int e = bk.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    int k = bk.y;
    HaloEnt h = plan[e];
    f[pidx(G, L, h.dt, k) + h.di] = f[pidx(G, L, h.st, k) + h.si];
}

template <class T>
DEVI void k_halo_pair(Bk bk, Geo G, const HaloEnt *__restrict__ plan, int count, T *fx, T *fy, int L)
{
    int e = bk.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    int k = bk.y;
    HaloEnt h = plan[e];
    const T *src = (h.sel & 1) ? fy : fx;
    T *dst = (h.sel & 4) ? fy : fx;
    T v = src[pidx(G, L, h.st, k) + h.si];
    dst[pidx(G, L, h.dt, k) + h.di] = (h.sel & 2) ? -v : v;
}

// up to four fields of one type and level count in one launch: grid y runs
// over (field, level)
template <class T>
struct FieldSet {
    T *p[4];
};
template <class T>
DEVI void k_halo_set(Bk bk, Geo G, const HaloEnt *__restrict__ plan, int count, FieldSet<T> F, int L)
{
    int e = bk.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    int q = (int)bk.y / L, k = (int)bk.y % L;
    T *f = q == 0 ? F.p[0] : q == 1 ? F.p[1] : q == 2 ? F.p[2] : F.p[3];
    HaloEnt h = plan[e];
    f[pidx(G, L, h.dt, k) + h.di] = f[pidx(G, L, h.st, k) + h.si];
}
template <class T>
static void halo_set(const fv3_grid *g, FieldSet<T> F, int nf, int L, hipStream_t st)
{
    if (g->planC.count == 0) return;
    launch_fn<k_halo_set<T>>("k_halo_scalar", dim3((g->planC.count + 255) / 256, L * nf), dim3(256), st,
                 g->geo, (const HaloEnt *)g->planC.d, g->planC.count, F, L);
}

template <class T>
static void halo_scalar(const fv3_grid *g, T *f, int L, hipStream_t st)
{
    if (g->planC.count == 0) return;
    launch_fn<k_halo_scalar<T>>("k_halo_scalar", dim3((g->planC.count + 255) / 256, L), dim3(256), st,
                 g->geo, (const HaloEnt *)g->planC.d, g->planC.count, f, L);
}
// corner (B-grid) scalar field
template <class T>
static void halo_corner(const fv3_grid *g, T *f, int L, hipStream_t st)
{
    if (g->planB.count == 0) return;
    launch_fn<k_halo_scalar<T>>("k_halo_corner", dim3((g->planB.count + 255) / 256, L), dim3(256), st,
                 g->geo, (const HaloEnt *)g->planB.d, g->planB.count, f, L);
}
template <class T>
static void halo_pair(const fv3_grid *g, const Plan &p, T *fx, T *fy, int L, hipStream_t st)
{
    if (p.count == 0) return;
    launch_fn<k_halo_pair<T>>("k_halo_pair", dim3((p.count + 255) / 256, L), dim3(256), st, g->geo,
                 (const HaloEnt *)p.d, p.count, fx, fy, L);
}

// ====================================================================
// c_sw (half step dt2 on one level): D -> A -> C interpolation, upwind
// half-step cell fluxes, kinetic energy, corner vorticity, C-grid winds.
// ====================================================================
// --------------------------------------------------------------------
// c_sw fused: one launch per level for the whole half step.  A tile of
// CTX x CTY points (point (i, j) = cell (i, j), its west x-face and south
// y-face, its SW corner) over i, j in [-1, n + 1] stages in LDS the A-grid
// winds (cells i0-3..i0+CTX+1), delp, pt, w (cells i0-2..i0+CTX), then the
// C-grid face quantities, the half-step kinetic energy and the corner
// vorticity, and writes only what later stages read: uc, vc, delpc, ptc,
// wc and the area fluxes ax, ay.  Each block writes the outputs of its own
// points.  Corner-block reads follow the same corner views as the
// per-stage kernels; a view source outside the staged region is read (or,
// for the A-grid winds, recomputed) from global memory.
// --------------------------------------------------------------------
// Tile width: the points i in [-1, n + 1] split into ceil((n + 3) / CTX)
// tiles from i = -1; 33 covers C192's 195 points in 6 tiles (32 needed 7, the
// last with 3 useful columns: a mostly empty tile still issues every
// instruction of the kernel).
#ifndef FV3_CSW_CTX
#define FV3_CSW_CTX 33
#endif
constexpr int CTX = FV3_CSW_CTX, CNT = 256;
// layers per c_sw block (the block's 2-D metric terms stay in registers)
#ifndef FV3_CSW_LEVELS
#define FV3_CSW_LEVELS 4
#endif
constexpr int CSL = FV3_CSW_LEVELS;
// tile rows per precision: the FP64 tile is shorter so that its LDS allows
// five blocks per CU
template <class B>
struct CswRows {
    static constexpr int Y = 8;
};
template <>
struct CswRows<double> {
    static constexpr int Y = 4;
};

// A-grid winds at a cell from the D-grid winds; CORNER = false for blocks
// whose reads cannot reach a cube corner block (no view checks)
// One-sided stencils at cube tile edges (option edge_interp).  Along a
// sweep with tile edges at the interfaces 0 and n, the four points a, b, c,
// d are the stencil of the centred interpolation; where it would reach
// across an edge, the quadratic through the three nearest points on the own
// side (3/8, 3/4, -1/8 from the point next to the edge), and on the edge the
// mean of the two linear extrapolations of the two nearest points per side.
// cell_pt: centre of cell m from the interfaces m-1 .. m+2 (D -> A);
// face_pt: interface m from the centres m-2 .. m+1 (A -> C).
template <class B>
DEVI B cell_pt(B a, B b, B c, B d, int m, int n, bool edge)
{
    if (edge) {
        if (m == 0 || m == n) return (B)0.375 * b + (B)0.75 * c - (B)0.125 * d;
        if (m == -1 || m == n - 1) return (B)0.375 * c + (B)0.75 * b - (B)0.125 * a;
    }
    return (-a + (B)9 * b + (B)9 * c - d) / (B)16;
}
template <class B>
DEVI B face_pt(B a, B b, B c, B d, int m, int n, bool edge)
{
    if (edge) {
        if (m == 0 || m == n) return (B)0.75 * (b + c) - (B)0.25 * (a + d);
        if (m == 1 || m == n + 1) return (B)0.375 * b + (B)0.75 * c - (B)0.125 * d;
        if (m == -1 || m == n - 1) return (B)0.375 * c + (B)0.75 * b - (B)0.125 * a;
    }
    return (-a + (B)9 * b + (B)9 * c - d) / (B)16;
}

// the sweep of ua runs along j in column i, that of va along i in row j;
// the edge rule applies on sweeps whose cross index lies inside the tile
template <class B, bool CORNER, bool EI = false>
DEVI B ua_at(const Geo &G, const B *U, const B *V, int i, int j)
{
    B a, b, c, d;
    if constexpr (CORNER) {
        a = pvx(G, U, V, SY, i, j - 1, 1, true), b = pvx(G, U, V, SY, i, j, 1, true);
        c = pvx(G, U, V, SY, i, j + 1, 1, true), d = pvx(G, U, V, SY, i, j + 2, 1, true);
    } else {
        a = AT(U, i, j - 1), b = AT(U, i, j), c = AT(U, i, j + 1), d = AT(U, i, j + 2);
    }
    return cell_pt(a, b, c, d, j, G.n, EI && i >= 0 && i < G.n);
}
template <class B, bool CORNER, bool EI = false>
DEVI B va_at(const Geo &G, const B *U, const B *V, int i, int j)
{
    B a, b, c, d;
    if constexpr (CORNER) {
        a = pvy(G, U, V, SX, i - 1, j, 0, true), b = pvy(G, U, V, SX, i, j, 0, true);
        c = pvy(G, U, V, SX, i + 1, j, 0, true), d = pvy(G, U, V, SX, i + 2, j, 0, true);
    } else {
        a = AT(V, i - 1, j), b = AT(V, i, j), c = AT(V, i + 1, j), d = AT(V, i + 2, j);
    }
    return cell_pt(a, b, c, d, i, G.n, EI && j >= 0 && j < G.n);
}

// LDS elements of one c_sw block
template <int CTY>
constexpr int csw_lds()
{
    return 2 * (CTY + 5) * (CTX + 5) + 3 * (CTY + 3) * (CTX + 3) + 8 * (CTY + 2) * (CTX + 2) + 2 * (CTY + 1) * (CTX + 1);
}

// The 2-D metric terms a c_sw thread uses in phases 2-4, the same on every
// layer: loaded once per block into registers and kept for all its layers
// (the same threads own the same points on every layer).
template <class B>
struct CswMet {
    static constexpr int CTY = CswRows<B>::Y, HF = CTY + 2, WF = CTX + 2, HK = CTY + 1, WK = CTX + 1;
    static constexpr int N2 = (HF * WF + CNT - 1) / CNT, N3 = (HK * WK + CNT - 1) / CNT, N4 = (CTX * CTY + CNT - 1) / CNT;
    B cu2[N2], su2[N2], dy2[N2], cv2[N2], sv2[N2], dx2[N2];                            // C-grid faces
    B rs2[N3], ca[N3], ra[N3], dxs[N3], dxn[N3], dyw[N3], dye[N3], fb[N3], rac[N3];    // cells, corners
    B cu4[N4], su4[N4], rdx4[N4], cv4[N4], sv4[N4], rdy4[N4];                          // own faces
};
template <class B>
DEVI void csw_metrics(const Geo &G, const Mets<B> &M, const int t, const int i0, const int j0, CswMet<B> &Q)
{
    using Q_ = CswMet<B>;
    constexpr int CTY = Q_::CTY, HF = Q_::HF, WF = Q_::WF, HK = Q_::HK, WK = Q_::WK;
    const int n = G.n, tid = threadIdx.x;
#pragma unroll
    for (int m = 0; m < Q_::N2; m++) {
        const int e = tid + m * CNT, r = e / WF, c = e - r * WF;
        const int i = i0 - 1 + c, j = j0 - 1 + r;
        const bool in = e < HF * WF;
        const bool xf = in && (j >= -1 && j <= n) && ((j >= 0 && j < n) ? (i >= -1 && i <= n + 1) : (i >= 0 && i <= n));
        const bool yf = in && (i >= -1 && i <= n) && ((i >= 0 && i < n) ? (j >= -1 && j <= n + 1) : (j >= 0 && j <= n));
        Q.cu2[m] = xf ? AT(MP(M, M_COS_U), i, j) : (B)0;
        Q.su2[m] = xf ? AT(MP(M, M_RSIN_U), i, j) : (B)0;
        Q.dy2[m] = xf ? AT(MP(M, M_DY), i, j) : (B)0;
        Q.cv2[m] = yf ? AT(MP(M, M_COS_V), i, j) : (B)0;
        Q.sv2[m] = yf ? AT(MP(M, M_RSIN_V), i, j) : (B)0;
        Q.dx2[m] = yf ? AT(MP(M, M_DX), i, j) : (B)0;
    }
#pragma unroll
    for (int m = 0; m < Q_::N3; m++) {
        const int e = tid + m * CNT, r = e / WK, c = e - r * WK;
        const bool in = e < HK * WK;
        // cell (i0 - 1 + c, j0 - 1 + r) of the half-step update, corner (i0 + c, j0 + r)
        const int i = i0 - 1 + c, j = j0 - 1 + r, ic = i0 + c, jc = j0 + r;
        const bool cross = in && i >= -1 && i <= n && j >= -1 && j <= n && ((i >= 0 && i < n) || (j >= 0 && j < n));
        const bool mine = cross && i >= i0 && j >= j0;
        const bool corner = in && ic >= 0 && ic <= n && jc >= 0 && jc <= n;
        Q.rs2[m] = cross ? AT(MP(M, M_RSIN2_A), i, j) : (B)0;
        Q.ca[m] = cross ? AT(MP(M, M_COS_A), i, j) : (B)0;
        Q.ra[m] = mine ? AT(MP(M, M_RAREA), i, j) : (B)0;
        Q.dxs[m] = corner ? AT(MP(M, M_DXC), ic, jc - 1) : (B)0;
        Q.dxn[m] = corner ? AT(MP(M, M_DXC), ic, jc) : (B)0;
        Q.dyw[m] = corner ? AT(MP(M, M_DYC), ic - 1, jc) : (B)0;
        Q.dye[m] = corner ? AT(MP(M, M_DYC), ic, jc) : (B)0;
        Q.fb[m] = corner ? AT(MP(M, M_FB), ic, jc) : (B)0;
        Q.rac[m] = corner ? AT(MP(M, M_RAREA_C), ic, jc) : (B)0;
    }
#pragma unroll
    for (int m = 0; m < Q_::N4; m++) {
        const int e = tid + m * CNT, r = e / CTX, c = e - r * CTX;
        const int i = i0 + c, j = j0 + r;
        const bool in = e < CTX * CTY;
        const bool fu = in && i >= 0 && i <= n && j >= 0 && j < n, fv = in && i >= 0 && i < n && j >= 0 && j <= n;
        Q.cu4[m] = fu ? AT(MP(M, M_COS_U), i, j) : (B)0;
        Q.su4[m] = fu ? AT(MP(M, M_RSIN_U), i, j) : (B)0;
        Q.rdx4[m] = fu ? AT(MP(M, M_RDXC), i, j) : (B)0;
        Q.cv4[m] = fv ? AT(MP(M, M_COS_V), i, j) : (B)0;
        Q.sv4[m] = fv ? AT(MP(M, M_RSIN_V), i, j) : (B)0;
        Q.rdy4[m] = fv ? AT(MP(M, M_RDYC), i, j) : (B)0;
    }
}

template <class B, bool CORNER, bool EI>
DEVI void csw_body(Bk bk, B *L, const int t, const int k, const Geo &G, const CswMet<B> &Q, B dt2, const B *u,
                   const B *v, const B *delp, const B *pt, const B *w, B *uc, B *vc, B *delpc, B *ptc, B *wc,
                   B *ax, B *ay)
{
    constexpr int CTY = CswRows<B>::Y;
    constexpr int WA = CTX + 5, HA = CTY + 5;   // A-grid cells i0-3.., j0-3..
    constexpr int WD = CTX + 3, HD = CTY + 3;   // delp/pt/w cells i0-2.., j0-2..
    constexpr int WF = CTX + 2, HF = CTY + 2;   // faces i0-1.., j0-1..
    constexpr int WK = CTX + 1, HK = CTY + 1;   // ke cells i0-1..; vorticity corners i0..
    B *sUA = L, *sVA = sUA + HA * WA;
    B *sD = sVA + HA * WA, *sPT = sD + HD * WD, *sW = sPT + HD * WD;
    B *sUC = sW + HD * WD, *sFm = sUC + HF * WF, *sFp = sFm + HF * WF, *sFw = sFp + HF * WF;
    B *sVC = sFw + HF * WF, *sGm = sVC + HF * WF, *sGp = sGm + HF * WF, *sGw = sGp + HF * WF;
    B *sKE = sGw + HF * WF, *sVO = sKE + HK * WK;
    const int n = G.n;
    // the thread index is made opaque per layer, so that the compiler does
    // not hoist every layer-invariant index and address of the body out of
    // the block's layer loop into registers (it then needed all 256)
    int tid = threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    const int i0 = -1 + (int)bk.x * CTX, j0 = -1 + (int)bk.y * CTY;
    const long o = pidx(G, G.nz, t, k);
    const B *U = u + o, *V = v + o, *D = delp + o, *PT = pt + o, *Wf = w + o;

    auto inA = [&](int i, int j) { return i >= i0 - 3 && i <= i0 + CTX + 1 && j >= j0 - 3 && j <= j0 + CTY + 1; };
    auto aA = [&](int i, int j) { return (j - (j0 - 3)) * WA + (i - (i0 - 3)); };
    auto inD = [&](int i, int j) { return i >= i0 - 2 && i <= i0 + CTX && j >= j0 - 2 && j <= j0 + CTY; };
    auto aD = [&](int i, int j) { return (j - (j0 - 2)) * WD + (i - (i0 - 2)); };
    auto aF = [&](int i, int j) { return (j - (j0 - 1)) * WF + (i - (i0 - 1)); };
    auto aK = [&](int i, int j) { return (j - (j0 - 1)) * WK + (i - (i0 - 1)); };
    auto aV = [&](int i, int j) { return (j - j0) * WK + (i - i0); };

    // A-grid vector through the corner view (x / y component), from LDS
    // when the source cell is staged, else recomputed from the D-grid winds
    auto UAx = [&](int i, int j, int mode) -> B {
        if (CORNER && in_corner(G, SC, i, j)) {
            int qi, qj;
            bool cw;
            corner_src(G, SC, i, j, mode, qi, qj, cw);
            B val = inA(qi, qj) ? sVA[aA(qi, qj)] : va_at<B, true, EI>(G, U, V, qi, qj);
            return cw ? -val : val;
        }
        return sUA[aA(i, j)];
    };
    auto VAy = [&](int i, int j, int mode) -> B {
        if (CORNER && in_corner(G, SC, i, j)) {
            int qi, qj;
            bool cw;
            corner_src(G, SC, i, j, mode, qi, qj, cw);
            B val = inA(qi, qj) ? sUA[aA(qi, qj)] : ua_at<B, true, EI>(G, U, V, qi, qj);
            return !cw ? -val : val;
        }
        return sVA[aA(i, j)];
    };
    // cell scalar through the corner view
    auto cv = [&](const B *sArr, const B *gArr, int i, int j, int mode) -> B {
        if (CORNER && in_corner(G, SC, i, j)) {
            int qi, qj;
            bool cw;
            corner_src(G, SC, i, j, mode, qi, qj, cw);
            return inD(qi, qj) ? sArr[aD(qi, qj)] : AT(gArr, qi, qj);
        }
        return sArr[aD(i, j)];
    };

    // 1. A-grid winds and cell scalars (corner cells are not stored)
#pragma unroll
    for (int m = 0; m < (HA * WA + CNT - 1) / CNT; m++) {
        const int e = tid + m * CNT;
        if (e >= HA * WA) break;
        int r = e / WA, c = e - r * WA;
        int i = i0 - 3 + c, j = j0 - 3 + r;
        B a = 0, b = 0;
        const bool ok = i >= -3 && i <= n + 2 && j >= -3 && j <= n + 2;
        if constexpr (CORNER) {
            if (ok && !in_corner(G, SC, i, j)) {
                if (j >= -2 && j <= n + 1) a = ua_at<B, CORNER, EI>(G, U, V, i, j);
                if (i >= -2 && i <= n + 1) b = va_at<B, CORNER, EI>(G, U, V, i, j);
            }
        } else {
            // loads at clamped points (inside the planes), then select: no
            // branches around the loads
            const bool oka = ok && j >= -2 && j <= n + 1, okb = ok && i >= -2 && i <= n + 1;
            const int ic = min(max(i, -3), n + 2), jc = min(max(j, -3), n + 2);
            a = ua_at<B, false, EI>(G, U, V, ic, min(max(jc, -2), n + 1));
            b = va_at<B, false, EI>(G, U, V, min(max(ic, -2), n + 1), jc);
            a = oka ? a : (B)0;
            b = okb ? b : (B)0;
        }
        sUA[e] = a;
        sVA[e] = b;
    }
#pragma unroll
    for (int m = 0; m < (HD * WD + CNT - 1) / CNT; m++) {
        const int e = tid + m * CNT;
        if (e >= HD * WD) break;
        int r = e / WD, c = e - r * WD;
        int i = i0 - 2 + c, j = j0 - 2 + r;
        B a = 0, b = 0, c2 = 0;
        const bool ok = i >= -3 && i <= n + 2 && j >= -3 && j <= n + 2;
        if constexpr (CORNER) {
            if (ok && !in_corner(G, SC, i, j)) {
                a = AT(D, i, j);
                b = AT(PT, i, j);
                c2 = AT(Wf, i, j);
            }
        } else {
            const int ic = min(max(i, -3), n + 2), jc = min(max(j, -3), n + 2);
            a = AT(D, ic, jc);
            b = AT(PT, ic, jc);
            c2 = AT(Wf, ic, jc);
            a = ok ? a : (B)0;
            b = ok ? b : (B)0;
            c2 = ok ? c2 : (B)0;
        }
        sD[e] = a;
        sPT[e] = b;
        sW[e] = c2;
    }
    // The D-grid winds at the faces of phases 2 and 4 are loaded one phase
    // ahead, before the barrier that ends the previous phase (the 2-D metric
    // terms of every phase are in registers for all layers of the block).
    auto xface = [&](int i, int j) {
        return (j >= -1 && j <= n) && ((j >= 0 && j < n) ? (i >= -1 && i <= n + 1) : (i >= 0 && i <= n));
    };
    auto yface = [&](int i, int j) {
        return (i >= -1 && i <= n) && ((i >= 0 && i < n) ? (j >= -1 && j <= n + 1) : (j >= 0 && j <= n));
    };
    constexpr int N2 = CswMet<B>::N2, N4 = CswMet<B>::N4;
    B q2V[N2], q2U[N2];
#pragma unroll
    for (int m = 0; m < N2; m++) {
        const int e = tid + m * CNT, r = e / WF, c = e - r * WF;
        const int i = i0 - 1 + c, j = j0 - 1 + r;
        const bool in = e < HF * WF, xf = in && xface(i, j), yf = in && yface(i, j);
        const int ic = min(max(i, -3), n + 2), jc = min(max(j, -3), n + 2);   // inside the planes
        const B vv = AT(V, ic, jc), uu = AT(U, ic, jc);
        q2V[m] = xf ? vv : (B)0;
        q2U[m] = yf ? uu : (B)0;
    }
    __syncthreads();
    // 2. C-grid faces: winds before the update, area fluxes, upwind fluxes
#pragma unroll
    for (int m = 0; m < (HF * WF + CNT - 1) / CNT; m++) {
        const int e = tid + m * CNT;
        if (e >= HF * WF) break;
        int r = e / WF, c = e - r * WF;
        int i = i0 - 1 + c, j = j0 - 1 + r;
        bool own = i >= i0 && i < i0 + CTX && j >= j0 && j < j0 + CTY;
        bool xf = xface(i, j), yf = yface(i, j);
        // blocks without corner views compute every face and select (all their
        // LDS reads stay inside the tile); only the global stores are masked
        B uc0 = 0, fm = 0, fp = 0, fw = 0;
        if (CORNER ? xf : true) {
            B a = UAx(i - 2, j, 0), b = UAx(i - 1, j, 0), c1 = UAx(i, j, 0), d = UAx(i + 1, j, 0);
            uc0 = face_pt(a, b, c1, d, i, n, EI && j >= 0 && j < n);
            B fl = dt2 * (uc0 - q2V[m] * Q.cu2[m]) * Q.su2[m] * Q.dy2[m];
            int up = fl > 0 ? i - 1 : i;
            fm = fl * cv(sD, D, up, j, 0);
            fp = fm * cv(sPT, PT, up, j, 0);
            fw = fm * cv(sW, Wf, up, j, 0);
            if (own && xf) AT(ax + o, i, j) = fl;
            if (!xf) uc0 = fm = fp = fw = (B)0;
        }
        sUC[e] = uc0;
        sFm[e] = fm;
        sFp[e] = fp;
        sFw[e] = fw;
        B vc0 = 0, gm = 0, gp = 0, gw = 0;
        if (CORNER ? yf : true) {
            B a = VAy(i, j - 2, 1), b = VAy(i, j - 1, 1), c1 = VAy(i, j, 1), d = VAy(i, j + 1, 1);
            vc0 = face_pt(a, b, c1, d, j, n, EI && i >= 0 && i < n);
            B fl = dt2 * (vc0 - q2U[m] * Q.cv2[m]) * Q.sv2[m] * Q.dx2[m];
            int up = fl > 0 ? j - 1 : j;
            gm = fl * cv(sD, D, i, up, 1);
            gp = gm * cv(sPT, PT, i, up, 1);
            gw = gm * cv(sW, Wf, i, up, 1);
            if (own && yf) AT(ay + o, i, j) = fl;
            if (!yf) vc0 = gm = gp = gw = (B)0;
        }
        sVC[e] = vc0;
        sGm[e] = gm;
        sGp[e] = gp;
        sGw[e] = gw;
    }
    __syncthreads();
    // 3. half-step cells (own points) and kinetic energy (one ring wider);
    //    absolute vorticity at the corners
#pragma unroll
    for (int m = 0; m < (HK * WK + CNT - 1) / CNT; m++) {
        const int e = tid + m * CNT;
        if (e >= HK * WK) break;
        int r = e / WK, c = e - r * WK;
        int i = i0 - 1 + c, j = j0 - 1 + r;
        bool cross = i >= -1 && i <= n && j >= -1 && j <= n && ((i >= 0 && i < n) || (j >= 0 && j < n));
        B kev = 0;
        if (CORNER ? cross : true) {
            B rs2 = Q.rs2[m], ca = Q.ca[m];
            B a = sUA[aA(i, j)], b = sVA[aA(i, j)];
            B uu = (a - b * ca) * rs2, vv = (b - a * ca) * rs2;
            kev = (B)0.5 * dt2 * (uu * (uu > 0 ? sUC[aF(i, j)] : sUC[aF(i + 1, j)]) +
                                  vv * (vv > 0 ? sVC[aF(i, j)] : sVC[aF(i, j + 1)]));
            if (cross && i >= i0 && j >= j0) {
                B rar = Q.ra[m];
                B dp = sD[aD(i, j)];
                B dc = dp + (sFm[aF(i, j)] - sFm[aF(i + 1, j)] + sGm[aF(i, j)] - sGm[aF(i, j + 1)]) * rar;
                B rdc = (B)1 / dc;
                AT(delpc + o, i, j) = dc;
                AT(ptc + o, i, j) =
                    (sPT[aD(i, j)] * dp + (sFp[aF(i, j)] - sFp[aF(i + 1, j)] + sGp[aF(i, j)] - sGp[aF(i, j + 1)]) * rar) * rdc;
                AT(wc + o, i, j) =
                    (sW[aD(i, j)] * dp + (sFw[aF(i, j)] - sFw[aF(i + 1, j)] + sGw[aF(i, j)] - sGw[aF(i, j + 1)]) * rar) * rdc;
            }
        }
        sKE[e] = cross ? kev : (B)0;
    }
#pragma unroll
    for (int m = 0; m < (HK * WK + CNT - 1) / CNT; m++) {
        const int e = tid + m * CNT;
        if (e >= HK * WK) break;
        int r = e / WK, c = e - r * WK;
        int i = i0 + c, j = j0 + r;
        B vo = 0;
        // outside [0, n]^2 the metric registers are zero, so vo is zero
        if (CORNER ? (i >= 0 && i <= n && j >= 0 && j <= n) : true) {
            B ws = 1, wn = 1, ww = 1, we = 1;
            if (CORNER && is_vertex(G, i, j)) {
                if (j == 0) ws = 0.5; else wn = 0.5;
                if (i == 0) ww = 0.5; else we = 0.5;
            }
            B circ = ws * sUC[aF(i, j - 1)] * Q.dxs[m] - wn * sUC[aF(i, j)] * Q.dxn[m] -
                     ww * sVC[aF(i - 1, j)] * Q.dyw[m] + we * sVC[aF(i, j)] * Q.dye[m];
            vo = Q.fb[m] + circ * Q.rac[m];
        }
        sVO[e] = vo;
    }
    B q4V[N4], q4U[N4];
#pragma unroll
    for (int m = 0; m < N4; m++) {
        const int e = tid + m * CNT, r = e / CTX, c = e - r * CTX;
        const int i = i0 + c, j = j0 + r;
        const bool in = e < CTX * CTY;
        const bool fu = in && i >= 0 && i <= n && j >= 0 && j < n, fv = in && i >= 0 && i < n && j >= 0 && j <= n;
        const int ic = min(max(i, -3), n + 2), jc = min(max(j, -3), n + 2);
        const B vv = AT(V, ic, jc), uu = AT(U, ic, jc);
        q4V[m] = fu ? vv : (B)0;
        q4U[m] = fv ? uu : (B)0;
    }
    __syncthreads();
    // 4. C-grid wind update on the interior faces of the own points
#pragma unroll
    for (int m = 0; m < (CTX * CTY + CNT - 1) / CNT; m++) {
        const int e = tid + m * CNT;
        if (e >= CTX * CTY) break;
        int r = e / CTX, c = e - r * CTX;
        int i = i0 + c, j = j0 + r;
        const bool fu = i >= 0 && i <= n && j >= 0 && j < n, fv = i >= 0 && i < n && j >= 0 && j <= n;
        if (CORNER ? fu : true) {
            B u0 = sUC[aF(i, j)];
            B fy1 = dt2 * (q4V[m] - u0 * Q.cu4[m]) * Q.su4[m];
            B vt = fy1 > 0 ? sVO[aV(i, j)] : sVO[aV(i, j + 1)];
            B un = u0 + fy1 * vt + (sKE[aK(i - 1, j)] - sKE[aK(i, j)]) * Q.rdx4[m];
            if (fu) AT(uc + o, i, j) = un;
        }
        if (CORNER ? fv : true) {
            B v0 = sVC[aF(i, j)];
            B fx1 = dt2 * (q4U[m] - v0 * Q.cv4[m]) * Q.sv4[m];
            B vt = fx1 > 0 ? sVO[aV(i, j)] : sVO[aV(i + 1, j)];
            B vn = v0 - fx1 * vt + (sKE[aK(i, j - 1)] - sKE[aK(i, j)]) * Q.rdy4[m];
            if (fv) AT(vc + o, i, j) = vn;
        }
    }
}

template <class B, bool EI = false>
DEVI void k_csw(Bk bk, Geo G, Mets<B> M, B dt2, const B *u, const B *v, const B *delp, const B *pt,
                const B *w, B *uc, B *vc, B *delpc, B *ptc, B *wc, B *ax, B *ay)
{
    // a block needs the corner views only if its reads (tile, staging halo
    // and the interpolation stencils around it) reach a cube corner block
    constexpr int CTY = CswRows<B>::Y;
    const int n = G.n;
    const int i0 = -1 + (int)bk.x * CTX, j0 = -1 + (int)bk.y * CTY;
    const bool nx = i0 - 6 < 0 || i0 + CTX + 5 > n, ny = j0 - 6 < 0 || j0 + CTY + 5 > n;
    __shared__ B L[csw_lds<CTY>()];
    const int nzb = (G.nz + CSL - 1) / CSL;
    const int t = (int)bk.z / nzb, k0 = ((int)bk.z % nzb) * CSL, k1 = k0 + CSL < G.nz ? k0 + CSL : G.nz;
    CswMet<B> Q;
    csw_metrics<B>(G, M, t, i0, j0, Q);
    if (G.cube && nx && ny) {
#pragma clang loop unroll(disable)
        for (int k = k0; k < k1; k++)
            csw_body<B, true, EI>(bk, L, t, k, G, Q, dt2, u, v, delp, pt, w, uc, vc, delpc, ptc, wc, ax, ay);
    } else if (EI && (nx || ny)) {
#pragma clang loop unroll(disable)
        for (int k = k0; k < k1; k++)
            csw_body<B, false, EI>(bk, L, t, k, G, Q, dt2, u, v, delp, pt, w, uc, vc, delpc, ptc, wc, ax, ay);
    } else {
#pragma clang loop unroll(disable)
        for (int k = k0; k < k1; k++)
            csw_body<B, false, false>(bk, L, t, k, G, Q, dt2, u, v, delp, pt, w, uc, vc, delpc, ptc, wc, ax, ay);
    }
}

#ifndef FV3_CSW_OCC
#define FV3_CSW_OCC 6
#endif
template <> constexpr int kocc<k_csw<float, false>> = FV3_CSW_OCC;
template <> constexpr int kocc<k_csw<float, true>> = FV3_CSW_OCC;

// ====================================================================
// Vertical column work (one thread per column, k marching in FP64).
// ====================================================================
DEVI double zs_at(const Geo &G, const double *phis, int t, int i, int j, int mode)
{
    if (!phis) return 0.0;
    const double *P = phis + pidx(G, 1, t, 0);
    return sv(G, P, SC, i, j, mode) / GRAV;
}

// dz_c and the equation-of-state passes of riem_solver_c run over the
// half-step cells i, j in [-1, n] flattened row by row (one thread per
// column, 256 per block, grid x ceil((n + 2)^2 / 256) per tile): with
// wavefronts aligned to the interior origin a row of n + 2 columns takes
// ceil((n + 2) / 64) + 1 wavefronts (four at C192, two of them a third full),
// and these walks are bound by their arithmetic, which a wavefront issues
// whatever its active lanes.  A flattened wavefront covers at most two row
// segments.  (The two light passes of the solve are bound by memory and keep
// the aligned rows.)
inline __host__ __device__ int sim1c_flat_blocks(int n) { return ((n + 2) * (n + 2) + 255) / 256; }

// dz_c: half-step interface heights by first-order upwind transport of the
// interface heights with layer-averaged area fluxes (top interface: top
// layer), advective form, surface fixed; output the half-step thicknesses.
template <class B>
DEVI void k_dzc(KARGS, Geo G, MetD M, const double *delz, const double *phis, const B *ax,
                      const B *ay, double *delzc)
{
    const int w = G.n + 2, p = (int)(bk.x * blockDim.x + threadIdx.x);
    if (p >= w * w) return;
    const int j = -1 + p / w, i = -1 + p % w;
    (void)ib; (void)ilo; (void)ihi; (void)jlo; (void)jhi;
    int n = G.n, nz = G.nz, t = bk.z;
    if (!((i >= 0 && i < n) || (j >= 0 && j < n))) return;
    double area = AT(MP(M, M_AREA), i, j);
    double zc = zs_at(G, phis, t, i, j, 0);
    double zw = zs_at(G, phis, t, i - 1, j, 0), ze = zs_at(G, phis, t, i + 1, j, 0);
    double zsou = zs_at(G, phis, t, i, j - 1, 1), znor = zs_at(G, phis, t, i, j + 1, 1);
    double zprev = zc;   // new height of the interface below
    // Walk bottom-up.  Level K needs the thicknesses of layer K at the cell
    // and its four neighbours and the area fluxes of layers K and K - 1 (the
    // interface mean); the layer K - 1 values are loaded one step ahead and
    // carried, so every value is loaded once and the next level's loads are
    // in flight while the current one computes.
    long o = pidx(G, nz, t, nz - 1);
    const double *D = delz + o;
    double dc = AT(D, i, j), dw = sv(G, D, SC, i - 1, j, 0), de = sv(G, D, SC, i + 1, j, 0);
    double ds = sv(G, D, SC, i, j - 1, 1), dn = sv(G, D, SC, i, j + 1, 1);
    double ax0 = (double)AT(ax + o, i, j), ax1 = (double)AT(ax + o, i + 1, j);
    double ay0 = (double)AT(ay + o, i, j), ay1 = (double)AT(ay + o, i, j + 1);
    for (int K = nz - 1; K >= 0; K--) {
        double ndc = 0, ndw = 0, nde = 0, nds = 0, ndn = 0, nax0 = 0, nax1 = 0, nay0 = 0, nay1 = 0;
        const long on = K > 0 ? pidx(G, nz, t, K - 1) : o;
        if (K > 0) {
            const double *Dn = delz + on;
            ndc = AT(Dn, i, j);
            ndw = sv(G, Dn, SC, i - 1, j, 0);
            nde = sv(G, Dn, SC, i + 1, j, 0);
            nds = sv(G, Dn, SC, i, j - 1, 1);
            ndn = sv(G, Dn, SC, i, j + 1, 1);
            nax0 = (double)AT(ax + on, i, j);
            nax1 = (double)AT(ax + on, i + 1, j);
            nay0 = (double)AT(ay + on, i, j);
            nay1 = (double)AT(ay + on, i, j + 1);
        }
        zc -= dc;
        zw -= dw;
        ze -= de;
        zsou -= ds;
        znor -= dn;
        double a0 = K == 0 ? ax0 : 0.5 * (nax0 + ax0);
        double a1 = K == 0 ? ax1 : 0.5 * (nax1 + ax1);
        double b0 = K == 0 ? ay0 : 0.5 * (nay0 + ay0);
        double b1 = K == 0 ? ay1 : 0.5 * (nay1 + ay1);
        double z0 = a0 > 0 ? zw : zc, z1 = a1 > 0 ? zc : ze;
        double y0 = b0 > 0 ? zsou : zc, y1 = b1 > 0 ? zc : znor;
        double zn = (zc * area + a0 * z0 - a1 * z1 + b0 * y0 - b1 * y1) / (area + a0 - a1 + b0 - b1);
        AT(delzc + o, i, j) = zprev - zn;
        zprev = zn;
        o = on;
        dc = ndc; dw = ndw; de = nde; ds = nds; dn = ndn;
        ax0 = nax0; ax1 = nax1; ay0 = nay0; ay1 = nay1;
    }
}

// Semi-implicit column solve (riem_solver_c / riem_solver3, Sec. IX-B):
// hydrostatic interface pressure from delp (top down), nonhydrostatic
// pressure from the equation of state, mass-weighted interface perturbation,
// backward-Euler tridiagonal system in w (Thomas), new perturbation by a
// top-down scan, thickness by inverting the equation of state, heights by a
// bottom-up scan.  Elimination coefficients live in FP64 scratch columns.
// The four passes are four launches (PASS = 1..4): one thread per column
// each, so that the light passes run at high occupancy and the two passes
// with the equation of state are not limited by the registers of the others.
// Every pass walks the column in groups of levels and issues the next
// group's loads before computing the current one.
#ifndef FV3_SIM1_SU
#define FV3_SIM1_SU 2
#endif
constexpr int SU = FV3_SIM1_SU;   // levels per prefetch group, passes 1 and 3
constexpr int SU2 = 8;            // levels per prefetch group, passes 2 and 4

// Moist column solves: the equation of state takes the virtual potential
// temperature theta (1 + (Rv/Rd - 1) q), q the specific humidity (none: dry).
constexpr double RVGAS = 461.5;
constexpr double EPSV = RVGAS / RDGAS - 1.0;
template <class B>
DEVI double virt(const B *qv, long o)
{
    return qv ? 1.0 + EPSV * (double)qv[o] : 1.0;
}

// Interface value at x = 0 of the cubic whose means over four consecutive
// layers of thicknesses da, db | dc, dd (the interface between db and dc)
// are qa, qb | qc, qd: the derivative at the middle node of the quartic
// through the cumulative contents at the five layer boundaries (Lagrange
// form, contents and nodes measured from the interface).  Exact for cubics.
DEVI double cubic_iface(double da, double db, double dc, double dd, double qa, double qb, double qc, double qd)
{
    const double x0 = -(da + db), x1 = -db, x3 = dc, x4 = dc + dd;
    const double Q0 = -(qa * da + qb * db), Q1 = -qb * db, Q3 = qc * dc, Q4 = qc * dc + qd * dd;
    const double l0 = -(x1 * x3 * x4) / ((x0 - x1) * x0 * (x0 - x3) * (x0 - x4));
    const double l1 = -(x0 * x3 * x4) / ((x1 - x0) * x1 * (x1 - x3) * (x1 - x4));
    const double l3 = -(x0 * x1 * x4) / ((x3 - x0) * (x3 - x1) * x3 * (x3 - x4));
    const double l4 = -(x0 * x1 * x3) / ((x4 - x0) * (x4 - x1) * x4 * (x4 - x3));
    return Q0 * l0 + Q1 * l1 + Q3 * l3 + Q4 * l4;
}

// SITE tells the two solves apart in profiles (0 riem_solver_c, 1 riem_solver3);
// OFFC: off-centred solve (beta < 1), a separate instantiation so that the
// backward-Euler passes keep their registers; PPO: interface perturbation
// (2 mass-linear, 4 cubic where two layers lie on each side; pass 1 only);
// MOIST: humidity in the equation of state (passes 1 and 3)
template <class B, class TW, int PASS, int SITE, bool OFFC = false, int PPO = 2, bool MOIST = false>
DEVI void k_sim1(KARGS, Geo G, double dt, double beta, double ptop, const B *dpi,
                                              const B *theta, const B *qv_, const double *delz, const TW *w,
                                              const double *phis, double *cpv, double *dpv,
                                              double *wnv, TW *w_out, double *delz_out,
                                              double *pfull, double *phi, int need_cross)
{
    int i, j;
    if constexpr (SITE == 0 && (PASS == 1 || PASS == 3)) {
        const int w = G.n + 2, p = (int)(bk.x * blockDim.x + threadIdx.x);
        if (p >= w * w) return;
        j = -1 + p / w;
        i = -1 + p % w;
    } else {
        i = ib + (int)(bk.x * blockDim.x + threadIdx.x);
        j = jlo + (int)(bk.y * blockDim.y + threadIdx.y);
        if (i < ilo || i > ihi || j > jhi) return;
    }
    int n = G.n, nz = G.nz, t = bk.z;
    if (need_cross && !((i >= 0 && i < n) || (j >= 0 && j < n))) return;
    const double kap = RDGAS / CP_AIR, gam = 1.0 / (1.0 - kap), rgam = 1.0 / gam;
    const long base = pidx(G, nz, t, 0) + (long)j * G.pitch + i, lev = G.lev;
    const long basei = pidx(G, nz + 1, t, 0) + (long)j * G.pitch + i;
    const double dt2x = dt * dt;
    // humidity only in the moist instantiation: the dry one folds the factor away
    const B *qv = MOIST ? qv_ : nullptr;
    // Each pass walks the column in groups of SU levels and issues the loads
    // of the next group before computing the current one, so that SU levels
    // of every input are in flight per thread (the column recurrences are
    // sequential; this is what hides HBM latency).
    struct G4 {
        double a[SU], b[SU], c[SU], d[SU], e[SU];   // e: humidity of the layer (0 when dry)
    };
    struct G2 {
        double a[SU2], b[SU2];
    };
    (void)dt2x;
    (void)rgam;

    // ---- pass 1: top-down elimination; step k consumes layer k + 1
    if constexpr (PASS == 1 && PPO == 2) {
    double lpi_k = flog(ptop);
    double dp0 = (double)dpi[base], th0 = (double)theta[base] * virt(qv, base), h0 = -delz[base], w0 = (double)w[base];
    double pi_k1 = ptop + dp0, lpi_k1 = flog(pi_k1);
    double m0 = dp0 / GRAV;
    double pp0 = P_REF * exp(gam * flog(RDGAS * th0 * m0 / (h0 * P_REF))) - dp0 / (lpi_k1 - lpi_k);
    double pps_k = 0.0, A_k = 0.0, cprev = 0.0, dprev = 0.0, wprev = 0.0;
    // off-centring: coupling scaled by beta^2, the explicit part of the
    // pressure response on the right-hand side; P* kept at the interfaces
    // (in the interface-pressure output) for pass 3
    const double bb = OFFC ? beta * beta : 1.0, ex = (1.0 - beta) / beta;
    {
        G4 cur, nxt;
#pragma unroll
        for (int u = 0; u < SU; u++) {
            int kk = 1 + u;
            long o = base + (long)kk * lev;
            bool in = kk < nz;
            cur.a[u] = in ? (double)dpi[o] : 0.0;
            cur.b[u] = in ? (double)theta[o] : 0.0;
            cur.e[u] = (in && qv) ? (double)qv[o] : 0.0;
            cur.c[u] = in ? -delz[o] : 0.0;
            cur.d[u] = in ? (double)w[o] : 0.0;
        }
        for (int k0 = 0; k0 < nz; k0 += SU) {
            if (k0 + SU < nz) {
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    int kk = k0 + SU + 1 + u;
                    long o = base + (long)kk * lev;
                    bool in = kk < nz;
                    nxt.a[u] = in ? (double)dpi[o] : 0.0;
                    nxt.b[u] = in ? (double)theta[o] : 0.0;
                    nxt.e[u] = (in && qv) ? (double)qv[o] : 0.0;
                    nxt.c[u] = in ? -delz[o] : 0.0;
                    nxt.d[u] = in ? (double)w[o] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < SU; u++) {
                int k = k0 + u;
                if (k < nz) {
                    double dp1 = cur.a[u], th1 = cur.b[u] * (1.0 + EPSV * cur.e[u]), h1 = cur.c[u], w1 = cur.d[u];
                    double pps_k1, A_k1, pi_k2 = 0, lpi_k2 = 0, m1 = 0, pp1 = 0;
                    if (k < nz - 1) {
                        pi_k2 = pi_k1 + dp1;
                        lpi_k2 = flog(pi_k2);
                        m1 = dp1 / GRAV;
                        pp1 = P_REF * exp(gam * flog(RDGAS * th1 * m1 / (h1 * P_REF))) - dp1 / (lpi_k2 - lpi_k1);
                        pps_k1 = (dp1 * pp0 + dp0 * pp1) / (dp0 + dp1);
                        A_k1 = bb * gam * (pi_k1 + pps_k1) * dt2x / (0.5 * (h0 + h1));
                    } else {
                        pps_k1 = pp0;
                        A_k1 = bb * gam * (pi_k1 + pps_k1) * dt2x / (0.5 * h0);
                    }
                    double lower = k > 0 ? -A_k : 0.0;
                    double diag = m0 + A_k + A_k1;
                    double upper = k < nz - 1 ? -A_k1 : 0.0;
                    double rhs = m0 * w0 + dt * (pps_k1 - pps_k);
                    if constexpr (OFFC) {
                        double wa = k > 0 ? wprev : 0.0, wb = k < nz - 1 ? w1 : 0.0;
                        rhs -= ex * (A_k1 * (w0 - wb) - A_k * (wa - w0));
                        pfull[basei + (long)(k + 1) * lev] = pps_k1;
                    }
                    double piv = diag - lower * cprev;
                    double rpiv = 1.0 / piv;
                    double ck = upper * rpiv;
                    double dk = (rhs - lower * dprev) * rpiv;
                    cpv[base + (long)k * lev] = ck;
                    dpv[base + (long)k * lev] = dk;
                    cprev = ck;
                    dprev = dk;
                    wprev = w0;
                    pi_k1 = pi_k2; lpi_k1 = lpi_k2; dp0 = dp1; m0 = m1; h0 = h1; pp0 = pp1; w0 = w1;
                    pps_k = pps_k1; A_k = A_k1;
                }
            }
            cur = nxt;
        }
    }
    }
    // ---- pass 1 with the cubic interface perturbation: step k consumes
    // layer k + 2 (its equation of state), so that the perturbations of the
    // layers k - 1 .. k + 2 around interface k + 1 are at hand
    if constexpr (PASS == 1 && PPO == 4) {
    const double bb = OFFC ? beta * beta : 1.0, ex = (1.0 - beta) / beta;
    double dp0 = (double)dpi[base], th0 = (double)theta[base] * virt(qv, base), h0 = -delz[base], w0 = (double)w[base];
    double pi1 = ptop + dp0, lpi1 = flog(pi1);
    double m0 = dp0 / GRAV;
    double pp0 = P_REF * exp(gam * flog(RDGAS * th0 * m0 / (h0 * P_REF))) - dp0 / (lpi1 - flog(ptop));
    double dp1 = 0.0, h1 = 0.0, w1 = 0.0, pp1 = 0.0, pi2 = 0.0, lpi2 = 0.0, m1 = 0.0;
    if (nz > 1) {
        const long o = base + lev;
        dp1 = (double)dpi[o];
        const double th1 = (double)theta[o] * virt(qv, o);
        h1 = -delz[o];
        w1 = (double)w[o];
        pi2 = pi1 + dp1;
        lpi2 = flog(pi2);
        m1 = dp1 / GRAV;
        pp1 = P_REF * exp(gam * flog(RDGAS * th1 * m1 / (h1 * P_REF))) - dp1 / (lpi2 - lpi1);
    }
    double dpm = 0.0, ppm = 0.0;   // layer k - 1
    double pps_k = 0.0, A_k = 0.0, cprev = 0.0, dprev = 0.0, wprev = 0.0;
    {
        G4 cur, nxt;
#pragma unroll
        for (int u = 0; u < SU; u++) {
            int kk = 2 + u;
            long o = base + (long)kk * lev;
            bool in = kk < nz;
            cur.a[u] = in ? (double)dpi[o] : 0.0;
            cur.b[u] = in ? (double)theta[o] : 0.0;
            cur.e[u] = (in && qv) ? (double)qv[o] : 0.0;
            cur.c[u] = in ? -delz[o] : 0.0;
            cur.d[u] = in ? (double)w[o] : 0.0;
        }
        for (int k0 = 0; k0 < nz; k0 += SU) {
            if (k0 + SU < nz) {
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    int kk = k0 + SU + 2 + u;
                    long o = base + (long)kk * lev;
                    bool in = kk < nz;
                    nxt.a[u] = in ? (double)dpi[o] : 0.0;
                    nxt.b[u] = in ? (double)theta[o] : 0.0;
                    nxt.e[u] = (in && qv) ? (double)qv[o] : 0.0;
                    nxt.c[u] = in ? -delz[o] : 0.0;
                    nxt.d[u] = in ? (double)w[o] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < SU; u++) {
                int k = k0 + u;
                if (k < nz) {
                    const double dp2 = cur.a[u], th2 = cur.b[u] * (1.0 + EPSV * cur.e[u]), h2 = cur.c[u], w2 = cur.d[u];
                    double pi3 = 0.0, lpi3 = 0.0, m2 = 0.0, pp2 = 0.0;
                    if (k + 2 < nz) {
                        pi3 = pi2 + dp2;
                        lpi3 = flog(pi3);
                        m2 = dp2 / GRAV;
                        pp2 = P_REF * exp(gam * flog(RDGAS * th2 * m2 / (h2 * P_REF))) - dp2 / (lpi3 - lpi2);
                    }
                    double pps_k1, A_k1;
                    if (k < nz - 1) {
                        if (k >= 1 && k <= nz - 3) pps_k1 = cubic_iface(dpm, dp0, dp1, dp2, ppm, pp0, pp1, pp2);
                        else pps_k1 = (dp1 * pp0 + dp0 * pp1) / (dp0 + dp1);
                        A_k1 = bb * gam * (pi1 + pps_k1) * dt2x / (0.5 * (h0 + h1));
                    } else {
                        pps_k1 = pp0;
                        A_k1 = bb * gam * (pi1 + pps_k1) * dt2x / (0.5 * h0);
                    }
                    double lower = k > 0 ? -A_k : 0.0;
                    double diag = m0 + A_k + A_k1;
                    double upper = k < nz - 1 ? -A_k1 : 0.0;
                    double rhs = m0 * w0 + dt * (pps_k1 - pps_k);
                    if constexpr (OFFC) {
                        double wa = k > 0 ? wprev : 0.0, wb = k < nz - 1 ? w1 : 0.0;
                        rhs -= ex * (A_k1 * (w0 - wb) - A_k * (wa - w0));
                        pfull[basei + (long)(k + 1) * lev] = pps_k1;
                    }
                    double piv = diag - lower * cprev;
                    double rpiv = 1.0 / piv;
                    double ck = upper * rpiv;
                    double dk = (rhs - lower * dprev) * rpiv;
                    cpv[base + (long)k * lev] = ck;
                    dpv[base + (long)k * lev] = dk;
                    cprev = ck;
                    dprev = dk;
                    wprev = w0;
                    dpm = dp0; ppm = pp0;
                    dp0 = dp1; m0 = m1; h0 = h1; pp0 = pp1; w0 = w1; pi1 = pi2;
                    dp1 = dp2; m1 = m2; h1 = h2; pp1 = pp2; w1 = w2; pi2 = pi3; lpi2 = lpi3;
                    pps_k = pps_k1; A_k = A_k1;
                }
            }
            cur = nxt;
        }
    }
    }
    // ---- pass 2: back substitution (bottom-up)
    if constexpr (PASS == 2) {
        double wv = 0.0;
        G2 cur, nxt;
#pragma unroll
        for (int u = 0; u < SU2; u++) {
            int kk = nz - 1 - u;
            long o = base + (long)kk * lev;
            cur.a[u] = kk >= 0 ? cpv[o] : 0.0;
            cur.b[u] = kk >= 0 ? dpv[o] : 0.0;
        }
        for (int k0 = nz - 1; k0 >= 0; k0 -= SU2) {
            if (k0 - SU2 >= 0) {
#pragma unroll
                for (int u = 0; u < SU2; u++) {
                    int kk = k0 - SU2 - u;
                    long o = base + (long)kk * lev;
                    nxt.a[u] = kk >= 0 ? cpv[o] : 0.0;
                    nxt.b[u] = kk >= 0 ? dpv[o] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < SU2; u++) {
                int k = k0 - u;
                if (k >= 0) {
                    wv = cur.b[u] - cur.a[u] * wv;
                    wnv[base + (long)k * lev] = wv;
                }
            }
            cur = nxt;
        }
    }
    // ---- pass 3: new perturbation (top down), thicknesses, interface pressure
    if constexpr (PASS == 3) {
        const double lpref = flog(P_REF);
        double ppn = 0.0, pnk = 0.0, pik = ptop, lpik = flog(ptop);
        if (pfull) pfull[basei] = ptop;
        G4 cur, nxt;
#pragma unroll
        for (int u = 0; u < SU; u++) {
            int kk = u;
            long o = base + (long)kk * lev;
            bool in = kk < nz;
            cur.a[u] = in ? (double)dpi[o] : 0.0;
            cur.b[u] = in ? (double)theta[o] : 0.0;
            cur.e[u] = (in && qv) ? (double)qv[o] : 0.0;
            cur.c[u] = in ? wnv[o] : 0.0;
            cur.d[u] = in ? (double)w[o] : 0.0;
        }
        for (int k0 = 0; k0 < nz; k0 += SU) {
            if (k0 + SU < nz) {
#pragma unroll
                for (int u = 0; u < SU; u++) {
                    int kk = k0 + SU + u;
                    long o = base + (long)kk * lev;
                    bool in = kk < nz;
                    nxt.a[u] = in ? (double)dpi[o] : 0.0;
                    nxt.b[u] = in ? (double)theta[o] : 0.0;
                    nxt.e[u] = (in && qv) ? (double)qv[o] : 0.0;
                    nxt.c[u] = in ? wnv[o] : 0.0;
                    nxt.d[u] = in ? (double)w[o] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < SU; u++) {
                int k = k0 + u;
                if (k < nz) {
                    double dp = cur.a[u], th = cur.b[u] * (1.0 + EPSV * cur.e[u]), wk = cur.c[u], wo = cur.d[u];
                    double m = dp / GRAV;
                    double pik1 = pik + dp, lpik1 = flog(pik1);
                    double pib = dp / (lpik1 - lpik);
                    // the scan gives the off-centred perturbation; the new one follows
                    double ppn1 = ppn + m * (wk - wo) / dt;
                    double pnk1 = ppn1;
                    if constexpr (OFFC) pnk1 = (ppn1 - (1.0 - beta) * pfull[basei + (long)(k + 1) * lev]) / beta;
                    double pn = pib + 0.5 * (pnk + pnk1);
                    double hn = RDGAS * th * m / P_REF * exp(rgam * (lpref - flog(pn)));
                    cpv[base + (long)k * lev] = hn;   // reuse as the new thickness
                    if (pfull) pfull[basei + (long)(k + 1) * lev] = pik1 + pnk1;
                    if (w_out) w_out[base + (long)k * lev] = (TW)wk;
                    ppn = ppn1;
                    pnk = pnk1;
                    pik = pik1;
                    lpik = lpik1;
                }
            }
            cur = nxt;
        }
    }
    // ---- pass 4: heights (bottom up)
    if constexpr (PASS == 4) {
        double z = phis ? phis[pidx(G, 1, t, 0) + (long)j * G.pitch + i] / GRAV : 0.0;
        if (phi) phi[basei + (long)nz * lev] = GRAV * z;
        double cur[SU2], nxt[SU2];
#pragma unroll
        for (int u = 0; u < SU2; u++) {
            int kk = nz - 1 - u;
            cur[u] = kk >= 0 ? cpv[base + (long)kk * lev] : 0.0;
        }
        for (int k0 = nz - 1; k0 >= 0; k0 -= SU2) {
            if (k0 - SU2 >= 0) {
#pragma unroll
                for (int u = 0; u < SU2; u++) {
                    int kk = k0 - SU2 - u;
                    nxt[u] = kk >= 0 ? cpv[base + (long)kk * lev] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < SU2; u++) {
                int k = k0 - u;
                if (k >= 0) {
                    double hn = cur[u];
                    z += hn;
                    if (phi) phi[basei + (long)k * lev] = GRAV * z;
                    if (delz_out) delz_out[base + (long)k * lev] = -hn;
                }
            }
#pragma unroll
            for (int u = 0; u < SU2; u++) cur[u] = nxt[u];
        }
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
// and geopotential; layer mass weights from delpc.  Each thread walks PGK
// consecutive layers of its point: the interface below one layer is the
// interface above the next, so its pressure and geopotential are carried
// instead of loaded again (the face metric too).
#ifndef FV3_PGK
#define FV3_PGK 4
#endif
constexpr int PGK = FV3_PGK;
template <class B>
DEVI void k_pgradc(KARGS, Geo G, MetD M, double dt2, const B *delpc, const double *pkc,
                         const double *gz, B *uc, B *vc)
{
    const int i = ib + (int)(bk.x * blockDim.x + threadIdx.x);
    const int j = jlo + (int)(bk.y * blockDim.y + threadIdx.y);
    if (i < ilo || i > ihi || j > jhi) return;
    const int n = G.n, nz = G.nz, nzb = (nz + PGK - 1) / PGK;
    const int t = (int)bk.z / nzb, k0 = ((int)bk.z % nzb) * PGK;
    const bool fx = j < n, fy = i < n;   // x-face (i, j) and y-face (i, j) of this point
    if (!fx && !fy) return;
    const double dxc = fx ? AT(MP(M, M_DXC), i, j) : 0.0, dyc = fy ? AT(MP(M, M_DYC), i, j) : 0.0;
    // cells W = (i - 1, j), C = (i, j), S = (i, j - 1) at the interface above the layer
    long oi = pidx(G, nz + 1, t, k0);
    double zW = 0, pW = 0, zS = 0, pS = 0;
    if (fx) { zW = AT(gz + oi, i - 1, j); pW = AT(pkc + oi, i - 1, j); }
    if (fy) { zS = AT(gz + oi, i, j - 1); pS = AT(pkc + oi, i, j - 1); }
    double zC = AT(gz + oi, i, j), pC = AT(pkc + oi, i, j);
    const int k1 = k0 + PGK < nz ? k0 + PGK : nz;
    for (int k = k0; k < k1; k++) {
        const long o = pidx(G, nz, t, k), o1 = pidx(G, nz + 1, t, k + 1);
        const B *D = delpc + o;
        double zW1 = 0, pW1 = 0, zS1 = 0, pS1 = 0;
        if (fx) { zW1 = AT(gz + o1, i - 1, j); pW1 = AT(pkc + o1, i - 1, j); }
        if (fy) { zS1 = AT(gz + o1, i, j - 1); pS1 = AT(pkc + o1, i, j - 1); }
        const double zC1 = AT(gz + o1, i, j), pC1 = AT(pkc + o1, i, j);
        const double dC = (double)AT(D, i, j);
        if (fx)
            AT(uc + o, i, j) += (B)pgf(dt2, dxc, (double)AT(D, i - 1, j), dC, zW, zW1, zC, zC1, pW, pW1, pC, pC1);
        if (fy)
            AT(vc + o, i, j) += (B)pgf(dt2, dyc, (double)AT(D, i, j - 1), dC, zS, zS1, zC, zC1, pS, pS1, pC, pC1);
        zW = zW1; pW = pW1; zS = zS1; pS = pS1; zC = zC1; pC = pC1;
    }
}

// ====================================================================
// fv_tp_2d (Sec. IX-C): Lin-Rood flux-form transport on one level, fused.
// A cell tile (32 x 16 in FP32, 32 x 8 in FP64) plus 3-point halo is staged
// in LDS in both sweep views; outer PPM fluxes, inner advective half updates, final averaged and
// weighted fluxes, then an epilogue that applies the flux divergence:
//   EPI_FLUX   write the fluxes only
//   EPI_DELP   write fluxes, accumulate them (mass fluxes, Courant numbers),
//              new delp = delp + div F / area
//   EPI_MASSW  mass-weighted update (q delp_old area + div F) / (delp_new area)
//   EPI_ADV    advective update (q area + div F) / (area + div of area fluxes)
//   EPI_TRACER (q dp1 area + div F) / (dp2 area)
// With `iface`, the Courant numbers and area fluxes of plane k are the mean
// of layers k-1 and k (plane 0: layer 0), for interface heights.
// ====================================================================
enum { EPI_FLUX = 0, EPI_DELP = 1, EPI_MASSW = 2, EPI_ADV = 3, EPI_TRACER = 4 };
// Cell tile per field precision (measured on MI355X at C192 x 79: the FP64
// tile is smaller so that four blocks fit a CU's LDS at 256 threads each).
constexpr int FNT = 256;
template <class T>
struct FvTile {
    static constexpr int X = 32, Y = 16;
};
template <>
struct FvTile<double> {
    static constexpr int X = 32, Y = 8;
};

template <class T, class C, class M>
struct FvArgs {
    const T *q;
    int Lq;
    const C *crx, *cry, *xfx, *yfx;
    int Lc, iface;
    const M *mx, *my;      // optional flux weights (mass fluxes)
    const T *area;         // area metric (type T)
    const T *dxa, *dya;    // cell widths along x and y (type T; tile-edge PPM)
    int epi;
    T *FX, *FY;            // flux outputs (may be null)
    int edges_only;        // write the flux outputs on tile-edge faces only
    T *qout;               // cell output, Lq levels
    const T *dold, *dnew;  // EPI_MASSW
    const double *dp1, *dp2;            // EPI_TRACER
    double *mfx, *mfy;     // EPI_DELP accumulators
    C *cxa, *cya;
};

// Loads and stores through a block-uniform base pointer and a 32-bit
// unsigned element offset (one VALU add per access instead of 64-bit
// address arithmetic).
template <class T>
DEVI T ldo(const T *base, unsigned e)
{
    return *(const T *)((const char *)base + e * (unsigned)sizeof(T));
}
template <class T>
DEVI void sto(T *base, unsigned e, T v)
{
    *(T *)((char *)base + e * (unsigned)sizeof(T)) = v;
}

template <class T, class C>
DEVI T ccr(const C *a, const C *a0, unsigned idx, int avg)
{
    if (avg) return (T)(0.5 * ((double)ldo(a0, idx) + (double)ldo(a, idx)));
    return (T)ldo(a, idx);
}

// The transport tile in LDS (one instance per block, shared by both
// instantiations of the body).
template <class T>
struct FvLds {
    static constexpr int FTX = FvTile<T>::X, FTY = FvTile<T>::Y;
    static constexpr int QW = FTX + 6, QH = FTY + 6;
    static constexpr int YW = FTX + 6, YH = FTY + 1;   // y-faces: cols i0-3..i0+FTX+2, rows j0..j0+FTY
    static constexpr int XW = FTX + 1, XH = FTY + 6;   // x-faces: cols i0..i0+FTX, rows j0-3..j0+FTY+2
    T sQ[QH * QW], sQy[QH * QW], sAR[QH * QW];
    T sCY[YH * YW], sYF[YH * YW], sFy[YH * YW];
    T sCX[XH * XW], sXF[XH * XW], sFx[XH * XW];
    T sQi[FTY * QW];                // cells: cols i0-3..i0+FTX+2, rows j0..j0+FTY-1
    T sQj[QH * FTX];                // cells: cols i0..i0+FTX-1, rows j0-3..j0+FTY+2
};

// CORNER: the block's staging window reaches a cube corner block (only
// blocks at the four corners of a tile), so its field reads go through the
// corner views; every other block reads the plane directly.
template <class T, class C, class M, int EPI, int ORD, int EDGE, bool CORNER>
DEVI void fvtp_body(Bk bk, const Geo &G, const FvArgs<T, C, M> &A, FvLds<T> &L)
{
    constexpr int FTX = FvTile<T>::X, FTY = FvTile<T>::Y;
    constexpr int QW = FvLds<T>::QW, QH = FvLds<T>::QH;
    constexpr int YW = FvLds<T>::YW, YH = FvLds<T>::YH;
    constexpr int XW = FvLds<T>::XW, XH = FvLds<T>::XH;
    constexpr int N4X = (FTY * XW + FNT - 1) / FNT, N4Y = (YH * FTX + FNT - 1) / FNT;
    constexpr int N5 = (FTY * FTX + FNT - 1) / FNT;
    T *sQ = L.sQ, *sQy = L.sQy, *sAR = L.sAR, *sCY = L.sCY, *sYF = L.sYF, *sFy = L.sFy;
    T *sCX = L.sCX, *sXF = L.sXF, *sFx = L.sFx, *sQi = L.sQi, *sQj = L.sQj;
    const int n = G.n, tid = threadIdx.x;
    const int i0 = bk.x * FTX, j0 = bk.y * FTY;
    const int t = bk.z / A.Lc, k = bk.z % A.Lc;
    // plane pointers (block-uniform); the staged ones are rebased to the
    // halo corner (-3, -3) so that every offset is a non-negative 32-bit value
    const int P = (int)G.pitch;
    const unsigned hb = 3u * (unsigned)P + 3u;   // rebase of the staging windows
    const T *Q = A.q + pidx(G, A.Lq, t, k);
    const long oc = pidx(G, A.Lc, t, k);
    const int avg = EPI == EPI_ADV && A.iface && k > 0;   // set only for the interface heights
    const long ob = avg ? pidx(G, A.Lc, t, k - 1) : oc;
    const T *AR = A.area + G.off0 + (long)t * G.lev;
    const T *DXA = EDGE ? A.dxa + G.off0 + (long)t * G.lev : nullptr;
    const T *DYA = EDGE ? A.dya + G.off0 + (long)t * G.lev : nullptr;
    const T *Qh = Q - hb, *ARh = AR - hb;
    const C *cryh = A.cry + oc - hb, *yfxh = A.yfx + oc - hb, *crxh = A.crx + oc - hb, *xfxh = A.xfx + oc - hb;
    const C *cry0h = A.cry + ob - hb, *yfx0h = A.yfx + ob - hb, *crx0h = A.crx + ob - hb, *xfx0h = A.xfx + ob - hb;
    const M *MX = A.mx ? A.mx + oc : nullptr, *MY = A.my ? A.my + oc : nullptr;
    using PT = typename std::conditional<EPI == EPI_TRACER, double, T>::type;

    // 0. per-thread prefetch of the global operands of phases 4 and 5, in
    //    their storage types (with the delp epilogue also the old values of
    //    the flux accumulators that phase 4 adds to: their loads would
    //    otherwise wait behind the previous face's stores)
    M wx[N4X], wy[N4Y];
    constexpr int NAX = EPI == EPI_DELP ? N4X : 1, NAY = EPI == EPI_DELP ? N4Y : 1;
    double amx[NAX], amy[NAY];
    C acx[NAX], acy[NAY];
    PT pa[N5], pb[N5];
#pragma unroll
    for (int m = 0; m < N4X; m++) {
        int e = tid + m * FNT, r = e / XW, c = e - r * XW;
        int i = i0 + c, j = j0 + r;
        const bool in = e < FTY * XW && i <= n && j < n;
        wx[m] = (MX && in) ? ldo(MX, (unsigned)(j * P + i)) : (M)0;
        if constexpr (EPI == EPI_DELP) {
            // the faces phase 4 writes: c < FTX, or the last face i == n
            const bool own = in && (c < FTX || i == n) && !(EDGE && edge_face(i, n));
            amx[m] = own ? ldo(A.mfx + oc, (unsigned)(j * P + i)) : 0.0;
            acx[m] = own ? ldo(A.cxa + oc, (unsigned)(j * P + i)) : (C)0;
        }
    }
#pragma unroll
    for (int m = 0; m < N4Y; m++) {
        int e = tid + m * FNT, r = e / FTX, c = e - r * FTX;
        int i = i0 + c, j = j0 + r;
        const bool in = e < YH * FTX && i < n && j <= n;
        wy[m] = (MY && in) ? ldo(MY, (unsigned)(j * P + i)) : (M)0;
        if constexpr (EPI == EPI_DELP) {
            const bool own = in && (r < FTY || j == n) && !(EDGE && edge_face(j, n));
            amy[m] = own ? ldo(A.mfy + oc, (unsigned)(j * P + i)) : 0.0;
            acy[m] = own ? ldo(A.cya + oc, (unsigned)(j * P + i)) : (C)0;
        }
    }
#pragma unroll
    for (int m = 0; m < N5; m++) {
        int e = tid + m * FNT, r = e / FTX, c = e - r * FTX;
        int i = i0 + c, j = j0 + r;
        bool in = e < FTY * FTX && i < n && j < n;
        unsigned ci = (unsigned)(j * P + i);
        pa[m] = (PT)0;
        pb[m] = (PT)0;
        if constexpr (EPI == EPI_MASSW) {
            if (in) {
                pa[m] = ldo(A.dold + oc, ci);
                pb[m] = ldo(A.dnew + oc, ci);
            }
        } else if constexpr (EPI == EPI_TRACER) {
            if (in) {
                pa[m] = ldo(A.dp1 + oc, ci);
                pb[m] = ldo(A.dp2 + oc, ci);
            }
        }
    }
    // 1. stage the field (both sweep views), the area, the Courant numbers and
    //    the area fluxes of the tile and its halo: every load of the thread
    //    is issued before the first LDS write, so that they are all in flight
    //    together
    {
        constexpr int NSQ = (QH * QW + FNT - 1) / FNT, NSY = (YH * YW + FNT - 1) / FNT;
        constexpr int NSX = (XH * XW + FNT - 1) / FNT;
        T qx[NSQ], qy[NSQ], qa[NSQ], cy[NSY], fy[NSY], cx[NSX], fx[NSX];
#pragma unroll
        for (int m = 0; m < NSQ; m++) {
            const int e = tid + m * FNT, r = e / QW, c = e - r * QW;
            const int i = i0 - 3 + c, j = j0 - 3 + r;
            T vx = 0, vy = 0, ar = 0;
            if (e < QH * QW && i <= n + 2 && j <= n + 2) {
                if (CORNER && in_corner(G, SC, i, j)) {
                    vx = sv(G, Q, SC, i, j, 0);
                    vy = sv(G, Q, SC, i, j, 1);
                } else {
                    const unsigned u = (unsigned)((j + 3) * P + (i + 3));
                    vx = vy = ldo(Qh, u);
                    ar = ldo(ARh, u);
                }
            }
            qx[m] = vx;
            qy[m] = vy;
            qa[m] = ar;
        }
#pragma unroll
        for (int m = 0; m < NSY; m++) {
            const int e = tid + m * FNT, r = e / YW, c = e - r * YW;
            const int i = i0 - 3 + c, j = j0 + r;
            T cr = 0, fl = 0;
            if (e < YH * YW && i <= n + 2 && j <= n) {
                const unsigned u = (unsigned)((j + 3) * P + (i + 3));
                cr = ccr<T>(cryh, cry0h, u, avg);
                fl = ccr<T>(yfxh, yfx0h, u, avg);
            }
            cy[m] = cr;
            fy[m] = fl;
        }
#pragma unroll
        for (int m = 0; m < NSX; m++) {
            const int e = tid + m * FNT, r = e / XW, c = e - r * XW;
            const int i = i0 + c, j = j0 - 3 + r;
            T cr = 0, fl = 0;
            if (e < XH * XW && i <= n && j <= n + 2) {
                const unsigned u = (unsigned)((j + 3) * P + (i + 3));
                cr = ccr<T>(crxh, crx0h, u, avg);
                fl = ccr<T>(xfxh, xfx0h, u, avg);
            }
            cx[m] = cr;
            fx[m] = fl;
        }
#pragma unroll
        for (int m = 0; m < NSQ; m++) {
            const int e = tid + m * FNT;
            if (e < QH * QW) {
                sQ[e] = qx[m];
                sQy[e] = qy[m];
                sAR[e] = qa[m];
            }
        }
#pragma unroll
        for (int m = 0; m < NSY; m++) {
            const int e = tid + m * FNT;
            if (e < YH * YW) {
                sCY[e] = cy[m];
                sYF[e] = fy[m];
            }
        }
#pragma unroll
        for (int m = 0; m < NSX; m++) {
            const int e = tid + m * FNT;
            if (e < XH * XW) {
                sCX[e] = cx[m];
                sXF[e] = fx[m];
            }
        }
    }
    __syncthreads();
    // 2. outer fluxes of the field (unrolled: the LDS reads of the next
    //    faces overlap the arithmetic of the current one)
#pragma unroll
    for (int m = 0; m < (YH * YW + FNT - 1) / FNT; m++) {
        const int e = tid + m * FNT;
        if (e >= YH * YW) break;
        int r = e / YW, c = e - r * YW;
        int i = i0 - 3 + c, j = j0 + r;
        T f = 0;
        if (i <= n + 2 && j <= n) {
            const T *col = sQy + r * QW + c;
            f = ppm_lds<QW, ORD>(col, sCY[e]);
        }
        sFy[e] = f;
    }
#pragma unroll
    for (int m = 0; m < (XH * XW + FNT - 1) / FNT; m++) {
        const int e = tid + m * FNT;
        if (e >= XH * XW) break;
        int r = e / XW, c = e - r * XW;
        int i = i0 + c, j = j0 - 3 + r;
        T f = 0;
        if (i <= n && j <= n + 2) {
            const T *row = sQ + r * QW + c;
            f = ppm_lds<1, ORD>(row, sCX[e]);
        }
        sFx[e] = f;
    }
    if constexpr (EDGE) {
        // faces with an edge cell upwind, on sweeps whose cross index lies
        // inside the tile (at most six per row or column): the one-sided
        // values replace the centred ones
        __syncthreads();
        for (int e = tid; e < XH * 6; e += FNT) {
            const int r = e / 6, i = edge_face_at(e - r * 6, n), c = i - i0, j = j0 - 3 + r;
            if (c < 0 || c >= XW || j < 0 || j >= n) continue;
            bool west;
            const int pe = edge_pe(i, n, west);
            const int f = r * XW + c;
            sFx[f] = ppm_edge<ORD>(sQ + r * QW + c, 1, DXA + j * P + i - 3, 1, sCX[f], pe, west);
        }
        for (int e = tid; e < YW * 6; e += FNT) {
            const int c = e / 6, j = edge_face_at(e - c * 6, n), r = j - j0, i = i0 - 3 + c;
            if (r < 0 || r >= YH || i < 0 || i >= n) continue;
            bool west;
            const int pe = edge_pe(j, n, west);
            const int f = r * YW + c;
            sFy[f] = ppm_edge<ORD>(sQy + r * QW + c, QW, DYA + (j - 3) * P + i, P, sCY[f], pe, west);
        }
    }
    __syncthreads();
    // 3. inner advective half updates
#pragma unroll
    for (int m = 0; m < (FTY * QW + FNT - 1) / FNT; m++) {
        const int e = tid + m * FNT;
        if (e >= FTY * QW) break;
        int r = e / QW, c = e - r * QW;
        int i = i0 - 3 + c, j = j0 + r;
        T v = 0;
        if (i <= n + 2 && j < n) {
            T ar = sAR[(r + 3) * QW + c];
            T y0 = sYF[r * YW + c], y1 = sYF[(r + 1) * YW + c];
            v = rdiv(sQ[(r + 3) * QW + c] * ar + y0 * sFy[r * YW + c] - y1 * sFy[(r + 1) * YW + c], ar + y0 - y1);
        }
        sQi[e] = v;
    }
#pragma unroll
    for (int m = 0; m < (QH * FTX + FNT - 1) / FNT; m++) {
        const int e = tid + m * FNT;
        if (e >= QH * FTX) break;
        int r = e / FTX, c = e - r * FTX;
        int i = i0 + c, j = j0 - 3 + r;
        T v = 0;
        if (i < n && j <= n + 2) {
            T ar = sAR[r * QW + c + 3];
            T x0 = sXF[r * XW + c], x1 = sXF[r * XW + c + 1];
            v = rdiv(sQ[r * QW + c + 3] * ar + x0 * sFx[r * XW + c] - x1 * sFx[r * XW + c + 1], ar + x0 - x1);
        }
        sQj[e] = v;
    }
    __syncthreads();
    // 4. final fluxes (in place over the outer fluxes)
    // am, ac: the old accumulator values of the face (delp epilogue)
    auto put_x = [&](int i, int c, int fi, int s, T fx, T wgt, double am, C ac) {
        const T F = (T)0.5 * (fx + sFx[s]) * wgt;
        sFx[s] = F;
        if (c < FTX || i == n) {
            if (A.FX && (!A.edges_only || i == 0 || i == n)) sto(A.FX + oc, (unsigned)fi, F);
            if (EPI == EPI_DELP) {
                sto(A.mfx + oc, (unsigned)fi, am + (double)F);
                sto(A.cxa + oc, (unsigned)fi, (C)(ac + (C)sCX[s]));
            }
        }
    };
    auto put_y = [&](int j, int r, int fi, int s, T fy, T wgt, double am, C ac) {
        const T F = (T)0.5 * (fy + sFy[s]) * wgt;
        sFy[s] = F;
        if (r < FTY || j == n) {
            if (A.FY && (!A.edges_only || j == 0 || j == n)) sto(A.FY + oc, (unsigned)fi, F);
            if (EPI == EPI_DELP) {
                sto(A.mfy + oc, (unsigned)fi, am + (double)F);
                sto(A.cya + oc, (unsigned)fi, (C)(ac + (C)sCY[s]));
            }
        }
    };
#pragma unroll
    for (int m = 0; m < N4X; m++) {
        int e = tid + m * FNT;
        if (e >= FTY * XW) break;
        int r = e / XW, c = e - r * XW;
        int i = i0 + c, j = j0 + r;
        if (i <= n && j < n && !(EDGE && edge_face(i, n))) {
            const int s = (r + 3) * XW + c;
            T fx = ppm_lds<1, ORD>(sQi + r * QW + c, sCX[s]);
            put_x(i, c, j * P + i, s, fx, A.mx ? (T)wx[m] : sXF[s], amx[EPI == EPI_DELP ? m : 0],
                  acx[EPI == EPI_DELP ? m : 0]);
        }
    }
    if constexpr (EDGE) {
        // the faces with an edge cell upwind, at most six per row
        for (int e = tid; e < FTY * 6; e += FNT) {
            const int r = e / 6, i = edge_face_at(e - r * 6, n), c = i - i0, j = j0 + r;
            if (c < 0 || c >= XW || j >= n) continue;
            const int fi = j * P + i, s = (r + 3) * XW + c;
            bool west;
            const int pe = edge_pe(i, n, west);
            T fx = ppm_edge<ORD>(sQi + r * QW + c, 1, DXA + j * P + i - 3, 1, sCX[s], pe, west);
            const bool own = EPI == EPI_DELP && (c < FTX || i == n);
            put_x(i, c, fi, s, fx, MX ? (T)ldo(MX, (unsigned)fi) : sXF[s],
                  own ? ldo(A.mfx + oc, (unsigned)fi) : 0.0, own ? ldo(A.cxa + oc, (unsigned)fi) : (C)0);
        }
    }
#pragma unroll
    for (int m = 0; m < N4Y; m++) {
        int e = tid + m * FNT;
        if (e >= YH * FTX) break;
        int r = e / FTX, c = e - r * FTX;
        int i = i0 + c, j = j0 + r;
        if (i < n && j <= n && !(EDGE && edge_face(j, n))) {
            const int s = r * YW + c + 3;
            T fy = ppm_lds<FTX, ORD>(sQj + r * FTX + c, sCY[s]);
            put_y(j, r, j * P + i, s, fy, A.my ? (T)wy[m] : sYF[s], amy[EPI == EPI_DELP ? m : 0],
                  acy[EPI == EPI_DELP ? m : 0]);
        }
    }
    if constexpr (EDGE) {
        // the faces with an edge cell upwind, at most six per column
        for (int e = tid; e < FTX * 6; e += FNT) {
            const int c = e / 6, j = edge_face_at(e - c * 6, n), r = j - j0, i = i0 + c;
            if (r < 0 || r >= YH || i >= n) continue;
            const int fi = j * P + i, s = r * YW + c + 3;
            bool west;
            const int pe = edge_pe(j, n, west);
            T fy = ppm_edge<ORD>(sQj + r * FTX + c, FTX, DYA + (j - 3) * P + i, P, sCY[s], pe, west);
            const bool own = EPI == EPI_DELP && (r < FTY || j == n);
            put_y(j, r, fi, s, fy, MY ? (T)ldo(MY, (unsigned)fi) : sYF[s],
                  own ? ldo(A.mfy + oc, (unsigned)fi) : 0.0, own ? ldo(A.cya + oc, (unsigned)fi) : (C)0);
        }
    }
    if constexpr (EPI == EPI_FLUX) return;
    __syncthreads();
    // 5. flux-divergence update of the cells of the tile
    const long oq = pidx(G, A.Lq, t, k);
#pragma unroll
    for (int m = 0; m < N5; m++) {
        int e = tid + m * FNT;
        if (e >= FTY * FTX) break;
        int r = e / FTX, c = e - r * FTX;
        int i = i0 + c, j = j0 + r;
        if (i >= n || j >= n) continue;
        int ci = j * P + i;
        T fw = sFx[(r + 3) * XW + c], fe = sFx[(r + 3) * XW + c + 1];
        T fs = sFy[r * YW + c + 3], fn = sFy[(r + 1) * YW + c + 3];
        T ar = sAR[(r + 3) * QW + c + 3];
        T qc = sQ[(r + 3) * QW + c + 3];
        T out;
        if constexpr (EPI == EPI_DELP) {
            out = qc + rdiv(fw - fe + fs - fn, ar);
        } else if constexpr (EPI == EPI_MASSW) {
            out = rdiv(qc * (T)pa[m] * ar + fw - fe + fs - fn, (T)pb[m] * ar);
        } else if constexpr (EPI == EPI_ADV) {
            T x0 = sXF[(r + 3) * XW + c], x1 = sXF[(r + 3) * XW + c + 1];
            T y0 = sYF[r * YW + c + 3], y1 = sYF[(r + 1) * YW + c + 3];
            out = rdiv(qc * ar + fw - fe + fs - fn, ar + x0 - x1 + y0 - y1);
        } else {
            out = (T)(((double)qc * pa[m] * (double)ar + (double)fw - (double)fe + (double)fs - (double)fn) /
                      (pb[m] * (double)ar));
        }
        sto(A.qout + oq, (unsigned)ci, out);
    }
}


template <class T, class C, class M, int EPI, int ORD, int EDGE>
DEVI void k_fvtp(Bk bk, Geo G, FvArgs<T, C, M> A)
{
    constexpr int FTX = FvTile<T>::X, FTY = FvTile<T>::Y;
    __shared__ FvLds<T> L;
    const int n = G.n, i0 = bk.x * FTX, j0 = bk.y * FTY;
    const bool corner = G.cube && (i0 - 3 < 0 || i0 + FTX + 2 >= n) && (j0 - 3 < 0 || j0 + FTY + 2 >= n);
    if (corner) fvtp_body<T, C, M, EPI, ORD, EDGE, true>(bk, G, A, L);
    else fvtp_body<T, C, M, EPI, ORD, EDGE, false>(bk, G, A, L);
}

template <class T, class C, class M, int ORD, int EDGE>
static void fvtp_order(const fv3_grid *g, int planes, const FvArgs<T, C, M> &a, hipStream_t st)
{
    static const char *names[] = {"k_fvtp_flux", "k_fvtp_delp", "k_fvtp_massw", "k_fvtp_adv", "k_fvtp_tracer"};
    constexpr int FTX = FvTile<T>::X, FTY = FvTile<T>::Y;
    dim3 grd((unsigned)((g->n + FTX - 1) / FTX), (unsigned)((g->n + FTY - 1) / FTY), (unsigned)planes);
    if constexpr (ORD == 7) {
        // the positive-definite order exists for the tracer transport only
        launch_fn<k_fvtp<T, C, M, EPI_TRACER, ORD, EDGE>>(names[EPI_TRACER], grd, dim3(FNT), st, g->geo, a);
    } else {
        switch (a.epi) {
        case EPI_FLUX: launch_fn<k_fvtp<T, C, M, EPI_FLUX, ORD, EDGE>>(names[a.epi], grd, dim3(FNT), st, g->geo, a); break;
        case EPI_DELP: launch_fn<k_fvtp<T, C, M, EPI_DELP, ORD, EDGE>>(names[a.epi], grd, dim3(FNT), st, g->geo, a); break;
        case EPI_MASSW: launch_fn<k_fvtp<T, C, M, EPI_MASSW, ORD, EDGE>>(names[a.epi], grd, dim3(FNT), st, g->geo, a); break;
        case EPI_ADV: launch_fn<k_fvtp<T, C, M, EPI_ADV, ORD, EDGE>>(names[a.epi], grd, dim3(FNT), st, g->geo, a); break;
        default: launch_fn<k_fvtp<T, C, M, EPI_TRACER, ORD, EDGE>>(names[a.epi], grd, dim3(FNT), st, g->geo, a); break;
        }
    }
}

template <class T, class C, class M, int EDGE>
static void fvtp_ord(const fv3_grid *g, int ord, int planes, const FvArgs<T, C, M> &a, hipStream_t st)
{
    switch (ord) {
    case 5: fvtp_order<T, C, M, 5, EDGE>(g, planes, a, st); break;
    case 6: fvtp_order<T, C, M, 6, EDGE>(g, planes, a, st); break;
    case 7: fvtp_order<T, C, M, 7, EDGE>(g, planes, a, st); break;
    default: fvtp_order<T, C, M, 8, EDGE>(g, planes, a, st); break;
    }
}

// the grid's PPM order applies to every transport of the call; the tracer
// transport takes hord_tr when that is set.  On the cube with edge_ppm the
// tile-edge instantiation runs, with the cell widths in the field's type.
template <class T, class C, class M>
static void fvtp(const fv3_grid *g, int planes, const FvArgs<T, C, M> &a, hipStream_t st)
{
    int ord = g->p.hord;
    if (a.epi == EPI_TRACER && g->p.hord_tr != 0) ord = g->p.hord_tr;
    if (g->p.edge_ppm && g->p.kind == FV3_GRID_CUBED_SPHERE) {
        FvArgs<T, C, M> b = a;
        if constexpr (std::is_same<T, double>::value) {
            b.dxa = g->met[M_DXA];
            b.dya = g->met[M_DYA];
        } else {
            b.dxa = g->metf[M_DXA];
            b.dya = g->metf[M_DYA];
        }
        fvtp_ord<T, C, M, 1>(g, ord, planes, b, st);
    } else {
        fvtp_ord<T, C, M, 0>(g, ord, planes, a, st);
    }
}

// ====================================================================
// d_sw (full step bdt on one level), around the fused transport
// ====================================================================
// Courant numbers and area fluxes from the contravariant half-step C-grid
// winds (partner component: four-point mean of the other C-grid wind).
// CORNER = false for blocks whose reads cannot reach a cube corner block
// (no view checks).
template <class B, bool CORNER>
DEVI void dsw_courant_body(const Geo &G, const Mets<B> &M, B bdt, const B *UC, const B *VC, long o, int t, int i, int j,
                           B *ut, B *vt, B *crx, B *cry, B *xfx, B *yfx, bool &bad)
{
    const int n = G.n;
    const B *dxa = MP(M, M_DXA), *dya = MP(M, M_DYA);
    if (i >= 0 && i <= n && j >= -3 && j <= n + 2) {
        B vb;
        if constexpr (CORNER)
            vb = (B)0.25 * (pvy(G, UC, VC, SY, i - 1, j, 0, true) + pvy(G, UC, VC, SY, i, j, 0, true) +
                            pvy(G, UC, VC, SY, i - 1, j + 1, 0, true) + pvy(G, UC, VC, SY, i, j + 1, 0, true));
        else
            vb = (B)0.25 * (AT(VC, i - 1, j) + AT(VC, i, j) + AT(VC, i - 1, j + 1) + AT(VC, i, j + 1));
        B su = AT(MP(M, M_SIN_U), i, j);
        B uu = rdiv(AT(UC, i, j) - vb * AT(MP(M, M_COS_U), i, j), su * su);
        int up = uu > 0 ? i - 1 : i;
        B da = CORNER ? pvx(G, dxa, dya, SC, up, j, 0, false) : AT(dxa, up, j);
        B cr = rdiv(bdt * uu, da);
        AT(ut + o, i, j) = uu;
        AT(crx + o, i, j) = cr;
        AT(xfx + o, i, j) = bdt * uu * su * AT(MP(M, M_DY), i, j);
        bad |= fabs((double)cr) > 1.0;
    }
    if (i >= -3 && i <= n + 2 && j >= 0 && j <= n) {
        B ub;
        if constexpr (CORNER)
            ub = (B)0.25 * (pvx(G, UC, VC, SX, i, j - 1, 1, true) + pvx(G, UC, VC, SX, i + 1, j - 1, 1, true) +
                            pvx(G, UC, VC, SX, i, j, 1, true) + pvx(G, UC, VC, SX, i + 1, j, 1, true));
        else
            ub = (B)0.25 * (AT(UC, i, j - 1) + AT(UC, i + 1, j - 1) + AT(UC, i, j) + AT(UC, i + 1, j));
        B sv_ = AT(MP(M, M_SIN_V), i, j);
        B vv = rdiv(AT(VC, i, j) - ub * AT(MP(M, M_COS_V), i, j), sv_ * sv_);
        int up = vv > 0 ? j - 1 : j;
        B da = CORNER ? pvy(G, dxa, dya, SC, i, up, 1, false) : AT(dya, i, up);
        B cr = rdiv(bdt * vv, da);
        AT(vt + o, i, j) = vv;
        AT(cry + o, i, j) = cr;
        AT(yfx + o, i, j) = bdt * vv * sv_ * AT(MP(M, M_DX), i, j);
        bad |= fabs((double)cr) > 1.0;
    }
}
template <class B>
DEVI void k_dsw_courant(KARGS, Geo G, Mets<B> M, B bdt, const B *uc, const B *vc, B *ut, B *vt,
                              B *crx, B *cry, B *xfx, B *yfx, int *flags)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    // the block's reads span its points +-1 in both directions; corner views
    // exist only outside [0, n - 1] in both
    const int i0 = ib + (int)(bk.x * blockDim.x) - 1, i1 = i0 + (int)blockDim.x + 1;
    const int j0 = jlo + (int)(bk.y * blockDim.y) - 1, j1 = j0 + (int)blockDim.y + 1;
    const bool corner = G.cube && (i0 < 0 || i1 >= G.n) && (j0 < 0 || j1 >= G.n);
    bool bad = false;
    if (corner) dsw_courant_body<B, true>(G, M, bdt, uc + o, vc + o, o, t, i, j, ut, vt, crx, cry, xfx, yfx, bad);
    else dsw_courant_body<B, false>(G, M, bdt, uc + o, vc + o, o, t, i, j, ut, vt, crx, cry, xfx, yfx, bad);
    if (bad) atomicOr(flags, 1);
}

// absolute vorticity at cells from the D-grid circulation, and the kinetic
// energy at corners (D-grid u upwinded along x and v along y by PPM with the
// corner displacements of the contravariant C-grid winds)
template <class B, int ORD>
DEVI void k_dsw_omke(KARGS, Geo G, Mets<B> M, B bdt, B d2, B dd, B damin, const B *u, const B *v,
                           const B *ut, const B *vt, const B *hd, B hc, B *om, B *ke)
{
    int i, j;
    if constexpr (sizeof(B) == 4) {
        // FP32 (bound by its arithmetic): launched over the range flattened
        // by rows, so that no wavefront is mostly idle at the range's ends
        const int w = ihi - ilo + 1, p = (int)(bk.x * blockDim.x + threadIdx.x);
        if (p >= w * (jhi - jlo + 1)) return;
        j = jlo + p / w;
        i = ilo + p % w;
    } else {
        i = ib + (int)(bk.x * blockDim.x + threadIdx.x);
        j = jlo + (int)(bk.y * blockDim.y + threadIdx.y);
        if (i < ilo || i > ihi || j > jhi) return;
    }
    const int t = (int)bk.z / G.nz, k = (int)bk.z % G.nz;
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const B *U = u + o, *V = v + o;
    const B *dx = MP(M, M_DX), *dy = MP(M, M_DY);
    if (!in_corner(G, SC, i, j) && i <= n + 2 && j <= n + 2)
        AT(om + o, i, j) = AT(MP(M, M_FC), i, j) + rdiv(AT(U, i, j) * AT(dx, i, j) - AT(U, i, j + 1) * AT(dx, i, j + 1) -
                                                         AT(V, i, j) * AT(dy, i, j) + AT(V, i + 1, j) * AT(dy, i + 1, j),
                                                     AT(MP(M, M_AREA), i, j));
    if (i >= 0 && i <= n && j >= 0 && j <= n) {
        B ub = (B)0.5 * bdt * (AT(ut + o, i, j - 1) + AT(ut + o, i, j));
        B vb = (B)0.5 * bdt * (AT(vt + o, i - 1, j) + AT(vt + o, i, j));
        B cu = rdiv(ub, AT(dx, ub > 0 ? i - 1 : i, j));
        B cv = rdiv(vb, AT(dy, i, vb > 0 ? j - 1 : j));
        B uu = ppm6<ORD>(AT(U, i - 3, j), AT(U, i - 2, j), AT(U, i - 1, j), AT(U, i, j), AT(U, i + 1, j), AT(U, i + 2, j), cu);
        B vv = ppm6<ORD>(AT(V, i, j - 3), AT(V, i, j - 2), AT(V, i, j - 1), AT(V, i, j), AT(V, i, j + 1), AT(V, i, j + 2), cv);
        B kev = (B)0.5 * (ub * uu + vb * vv);
        if (d2 > (B)0 || dd > (B)0) {
            // del-2 divergence damping: minus nu times the divergence of the
            // D-grid winds over the corner's dual cell (half weights next to
            // the missing cell at a cube vertex), nu = damin times d2, raised
            // by the Smagorinsky magnitude dd sqrt(DT^2 + DS^2) up to 0.2
            B ws = 1, wn = 1, ww = 1, we = 1;
            if (is_vertex(G, i, j)) {
                if (j == 0) ws = 0.5; else wn = 0.5;
                if (i == 0) ww = 0.5; else we = 0.5;
            }
            const B *dxc = MP(M, M_DXC), *dyc = MP(M, M_DYC);
            B rac = AT(MP(M, M_RAREA_C), i, j);
            B fe = we * AT(U, i, j) * AT(dyc, i, j), fw = ww * AT(U, i - 1, j) * AT(dyc, i - 1, j);
            B fn = wn * AT(V, i, j) * AT(dxc, i, j), fs = ws * AT(V, i, j - 1) * AT(dxc, i, j - 1);
            B c2 = d2;
            if (dd > (B)0) {
                // tension at the corner; shear of the stored cells around it
                B ten = (fe - fw - fn + fs) * rac, sh = 0;
                int cnt = 0;
                const B *ra = MP(M, M_RAREA);
                for (int cj = j - 1; cj <= j; cj++)
                    for (int ci = i - 1; ci <= i; ci++) {
                        if (in_corner(G, SC, ci, cj)) continue;
                        sh += (AT(V, ci + 1, cj) * AT(dy, ci + 1, cj) - AT(V, ci, cj) * AT(dy, ci, cj) +
                               AT(U, ci, cj + 1) * AT(dx, ci, cj + 1) - AT(U, ci, cj) * AT(dx, ci, cj)) *
                              AT(ra, ci, cj);
                        cnt++;
                    }
                sh /= (B)cnt;
                B cs = dd * sqrt(ten * ten + sh * sh);
                cs = cs < (B)0.2 ? cs : (B)0.2;
                c2 = cs > c2 ? cs : c2;
            }
            kev -= c2 * damin * (fe - fw + fn - fs) * rac;
        }
        // higher-order damping: hc = (-1)^(nord+1) nu_n times the divergence
        // after nord corner Laplacians
        if (hd) kev += hc * AT(hd + o, i, j);
        AT(ke + o, i, j) = kev;
    }
}

// Edge-flux fix-up on the cube, one thread per (cell next to a tile edge,
// level): each of the cell's faces on the edge takes the mean of our flux and
// the neighbour tile's copy (mapped onto our direction); the cell takes the
// difference.  After d_sw: mass fluxes FXm/FYm (delp), content fluxes of pt
// and w, the committed delp, pt, w and the mass-flux accumulators.
template <class B>
DEVI B edge_mean_delta(const Geo &G, const EdgeCell &c, int q, int k, const B *FX, const B *FY)
{
    const B *own = c.arr[q] == 0 ? FX : FY, *par = c.parr[q] == 0 ? FX : FY;
    const B fo = own[pidx(G, G.nz, c.t, k) + c.off[q]];
    const B fp = (B)c.spar[q] * par[pidx(G, G.nz, c.pt[q], k) + c.poff[q]];
    return (B)0.5 * (fo + fp) - fo;
}

// Tile-edge kinetic energy (edge_ppm): at the corners whose wind sweeps have
// an edge cell upwind (i or j in 0, 1, 2, n-2, n-1, n) the upwinded winds take
// the one-sided face values, the widths being the face lengths dx (dy); the
// difference from the centred values k_dsw_omke used is added to ke.  One
// thread per corner of the six lines of each direction (corners on both a
// column and a row line counted once), levels in y, tiles in z.
template <class B, int ORD>
DEVI void k_ke_edge(Bk bk, Geo G, Mets<B> M, B bdt, const B *u, const B *v, const B *ut, const B *vt, B *ke)
{
    const int n = G.n, e = (int)(bk.x * blockDim.x + threadIdx.x), k = (int)bk.y, t = (int)bk.z;
    int i, j;
    if (e < 6 * (n + 1)) {
        // the six edge columns of one row are neighbouring threads
        j = e / 6;
        i = edge_face_at(e - 6 * j, n);
    } else {
        const int e2 = e - 6 * (n + 1);
        if (e2 >= 6 * (n - 5)) return;
        const int q = e2 / (n - 5);
        i = 3 + e2 - q * (n - 5);
        j = edge_face_at(q, n);
    }
    const long o = pidx(G, G.nz, t, k);
    const B *U = u + o, *V = v + o;
    const B *dx = MP(M, M_DX), *dy = MP(M, M_DY);
    B d = 0;
    bool west;
    if (edge_face(i, n)) {
        const B ub = (B)0.5 * bdt * (AT(ut + o, i, j - 1) + AT(ut + o, i, j));
        const B cu = rdiv(ub, AT(dx, ub > 0 ? i - 1 : i, j));
        const int pe = edge_pe(i, n, west);
        const B ue = ppm_edge<ORD>(&AT(U, i - 3, j), 1, &AT(dx, i - 3, j), 1, cu, pe, west);
        const B uc = ppm6<ORD>(AT(U, i - 3, j), AT(U, i - 2, j), AT(U, i - 1, j), AT(U, i, j), AT(U, i + 1, j),
                               AT(U, i + 2, j), cu);
        d += ub * (ue - uc);
    }
    if (edge_face(j, n)) {
        const B vb = (B)0.5 * bdt * (AT(vt + o, i - 1, j) + AT(vt + o, i, j));
        const B cv = rdiv(vb, AT(dy, i, vb > 0 ? j - 1 : j));
        const int pe = edge_pe(j, n, west);
        const B ve = ppm_edge<ORD>(&AT(V, i, j - 3), (int)G.pitch, &AT(dy, i, j - 3), (int)G.pitch, cv, pe, west);
        const B vc = ppm6<ORD>(AT(V, i, j - 3), AT(V, i, j - 2), AT(V, i, j - 1), AT(V, i, j), AT(V, i, j + 1),
                               AT(V, i, j + 2), cv);
        d += vb * (ve - vc);
    }
    AT(ke + o, i, j) += (B)0.5 * d;
}

template <class B>
DEVI void k_edgefix_dsw(Bk bk, Geo G, const EdgeCell *__restrict__ cells, int count, const B *area,
                        const B *FXm, const B *FYm, const B *FXp, const B *FYp, const B *FXw, const B *FYw,
                        B *delp, B *pt, B *w, double *mfx, double *mfy)
{
    const int e = (int)(bk.x * blockDim.x + threadIdx.x);
    if (e >= count) return;
    const int k = (int)bk.y;
    const EdgeCell c = cells[e];
    B dM = 0, dP = 0, dW = 0;
    for (int q = 0; q < c.nf; q++) {
        const B em = edge_mean_delta(G, c, q, k, FXm, FYm);
        dM += (B)c.sin[q] * em;
        dP += (B)c.sin[q] * edge_mean_delta(G, c, q, k, FXp, FYp);
        dW += (B)c.sin[q] * edge_mean_delta(G, c, q, k, FXw, FYw);
        double *acc = c.arr[q] == 0 ? mfx : mfy;
        acc[pidx(G, G.nz, c.t, k) + c.off[q]] += (double)em;
    }
    const long o = pidx(G, G.nz, c.t, k) + c.cell;
    const B a = area[pidx(G, 1, c.t, 0) + c.cell];
    const B d0 = delp[o], d1 = d0 + dM / a;
    pt[o] = (pt[o] * d0 * a + dP) / (d1 * a);
    w[o] = (w[o] * d0 * a + dW) / (d1 * a);
    delp[o] = d1;
}

// ... and after a tracer sub-cycle: tracer fluxes, the sub-cycle's new mass dp2.
template <class B>
DEVI void k_edgefix_q(Bk bk, Geo G, const EdgeCell *__restrict__ cells, int count, const B *area, const B *FX,
                      const B *FY, const double *dp2, B *qf)
{
    const int e = (int)(bk.x * blockDim.x + threadIdx.x);
    if (e >= count) return;
    const int k = (int)bk.y;
    const EdgeCell c = cells[e];
    B dQ = 0;
    for (int q = 0; q < c.nf; q++) dQ += (B)c.sin[q] * edge_mean_delta(G, c, q, k, FX, FY);
    const long o = pidx(G, G.nz, c.t, k) + c.cell;
    qf[o] = qf[o] + (B)((double)dQ / (dp2[o] * (double)area[pidx(G, 1, c.t, 0) + c.cell]));
}

// Divergence at corner (i, j) of a D-grid pair (U on y-faces, V on x-faces)
// over the corner's dual cell: normal components through its four edges
// times their lengths over the dual area, half weights for the two edges
// next to the missing cell at a cube vertex.
template <class B>
DEVI B corner_div_at(const Geo &G, const Mets<B> &M, const B *U, const B *V, int t, int i, int j)
{
    B ws = 1, wn = 1, ww = 1, we = 1;
    if (is_vertex(G, i, j)) {
        if (j == 0) ws = 0.5; else wn = 0.5;
        if (i == 0) ww = 0.5; else we = 0.5;
    }
    const B *dxc = MP(M, M_DXC), *dyc = MP(M, M_DYC);
    return (we * AT(U, i, j) * AT(dyc, i, j) - ww * AT(U, i - 1, j) * AT(dyc, i - 1, j) +
            wn * AT(V, i, j) * AT(dxc, i, j) - ws * AT(V, i, j - 1) * AT(dxc, i, j - 1)) *
           AT(MP(M, M_RAREA_C), i, j);
}

// Higher-order divergence damping: the corner divergence of the D-grid
// winds (corners 0..n of every level) ...
template <class B>
DEVI void k_cdiv(KARGS, Geo G, Mets<B> M, const B *u, const B *v, B *dg)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    AT(dg + o, i, j) = corner_div_at(G, M, u + o, v + o, t, i, j);
}

// ... and the corner Laplacian of a corner field whose halo is filled: the
// corner divergence of its gradient along the cell edges, (D(i+1,j) -
// D(i,j)) / dx on y-faces and (D(i,j+1) - D(i,j)) / dy on x-faces.
template <class B>
DEVI void k_clap(KARGS, Geo G, Mets<B> M, const B *d, B *out)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    const B *D = d + o, *rdx = MP(M, M_RDX), *rdy = MP(M, M_RDY);
    const B c = AT(D, i, j);
    const B ge = (AT(D, i + 1, j) - c) * AT(rdx, i, j), gw = (c - AT(D, i - 1, j)) * AT(rdx, i - 1, j);
    const B gn = (AT(D, i, j + 1) - c) * AT(rdy, i, j), gs = (c - AT(D, i, j - 1)) * AT(rdy, i, j - 1);
    B ws = 1, wn = 1, ww = 1, we = 1;
    if (is_vertex(G, i, j)) {
        if (j == 0) ws = 0.5; else wn = 0.5;
        if (i == 0) ww = 0.5; else we = 0.5;
    }
    const B *dxc = MP(M, M_DXC), *dyc = MP(M, M_DYC);
    AT(out + o, i, j) = (we * ge * AT(dyc, i, j) - ww * gw * AT(dyc, i - 1, j) + wn * gn * AT(dxc, i, j) -
                         ws * gs * AT(dxc, i, j - 1)) *
                        AT(MP(M, M_RAREA_C), i, j);
}

// D-grid wind update from kinetic-energy differences and vorticity fluxes;
// commit the transported delp, pt, w.
// Optional del-2 vorticity damping (nuv > 0): the diffusive flux of the
// relative vorticity (om - f) across each face joins the vorticity flux, so
// u gains nuv (w(i, j-1) - w(i, j)) / dyc and v loses nuv (w(i-1, j) - w(i, j)) / dxc.
template <class B>
DEVI void k_dsw_update(KARGS, Geo G, Mets<B> M, const B *ke, const B *VX, const B *VY,
                             const B *dn, const B *pn, const B *wn, const B *om, B nuv, B *u, B *v, B *delp,
                             B *pt, B *w)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const B *KE = ke + o;
    B du = 0, dv = 0;
    if (nuv > (B)0) {
        const B *OM = om + o, *fc = MP(M, M_FC);
        const B wc = AT(OM, i, j) - AT(fc, i, j);
        if (i < n) du = nuv * ((AT(OM, i, j - 1) - AT(fc, i, j - 1)) - wc) * AT(MP(M, M_RDYC), i, j);
        if (j < n) dv = -nuv * ((AT(OM, i - 1, j) - AT(fc, i - 1, j)) - wc) * AT(MP(M, M_RDXC), i, j);
    }
    if (i < n) AT(u + o, i, j) = AT(u + o, i, j) + (AT(KE, i, j) - AT(KE, i + 1, j) + AT(VY + o, i, j)) * AT(MP(M, M_RDX), i, j) + du;
    if (j < n) AT(v + o, i, j) = AT(v + o, i, j) + (AT(KE, i, j) - AT(KE, i, j + 1) - AT(VX + o, i, j)) * AT(MP(M, M_RDY), i, j) + dv;
    if (i < n && j < n) {
        AT(delp + o, i, j) = AT(dn + o, i, j);
        AT(pt + o, i, j) = AT(pn + o, i, j);
        AT(w + o, i, j) = AT(wn + o, i, j);
    }
}

// ====================================================================
// dz_d: interface heights transported by fv_tp_2d (EPI_ADV, interface
// averaged Courant numbers), surface fixed.
// ====================================================================
DEVI void k_heights(KARGS, Geo G, const double *delz, const double *phis, double *zh)
{
    int i = ib + (int)(bk.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(bk.y * blockDim.y + threadIdx.y);
    if (i < ilo || i > ihi || j > jhi) return;
    int nz = G.nz, t = bk.z;
    if (in_corner(G, SC, i, j)) return;
    long c = (long)j * G.pitch + i;
    double z = phis ? phis[pidx(G, 1, t, 0) + c] / GRAV : 0.0;
    zh[pidx(G, nz + 1, t, nz) + c] = z;
    for (int k = nz - 1; k >= 0; k--) {
        z -= delz[pidx(G, nz, t, k) + c];
        zh[pidx(G, nz + 1, t, k) + c] = z;
    }
}

// Mixed precision: the heights travel as FP32 deviations from a reference
// per (tile, interface), the height at cell (0, 0).  The transport is exactly
// translation-equivariant (PPM faces, advective inner and outer updates), so
// only the deviations' rounding enters, not that of the full height.  Every
// thread scans the reference column beside its own (the same loads for the
// whole tile, served by the cache); the thread of cell (0, 0) stores it.
DEVI void k_heights_dev(KARGS, Geo G, const double *delz, const double *phis, double *zref, float *zd)
{
    int i = ib + (int)(bk.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(bk.y * blockDim.y + threadIdx.y);
    if (i < ilo || i > ihi || j > jhi) return;
    int nz = G.nz, t = bk.z;
    if (in_corner(G, SC, i, j)) return;
    long c = (long)j * G.pitch + i;
    const bool keep = i == 0 && j == 0;
    double z = phis ? phis[pidx(G, 1, t, 0) + c] / GRAV : 0.0;
    double zr = phis ? phis[pidx(G, 1, t, 0)] / GRAV : 0.0;
    zd[pidx(G, nz + 1, t, nz) + c] = (float)(z - zr);
    if (keep) zref[t * (nz + 1) + nz] = zr;
    for (int k = nz - 1; k >= 0; k--) {
        z -= delz[pidx(G, nz, t, k) + c];
        zr -= delz[pidx(G, nz, t, k)];
        zd[pidx(G, nz + 1, t, k) + c] = (float)(z - zr);
        if (keep) zref[t * (nz + 1) + k] = zr;
    }
}

DEVI void k_delz_from_zdev(KARGS, Geo G, const float *zn, const double *zref, const double *phis, double *delz)
{
    KBEGIN(G.nz);
    int nz = G.nz;
    const double *zr = zref + t * (nz + 1);
    double top = zr[k] + (double)AT(zn + pidx(G, nz + 1, t, k), i, j);
    double below = k == nz - 1 ? (phis ? AT(phis + pidx(G, 1, t, 0), i, j) / GRAV : 0.0)
                               : zr[k + 1] + (double)AT(zn + pidx(G, nz + 1, t, k + 1), i, j);
    AT(delz + pidx(G, nz, t, k), i, j) = below - top;
}

DEVI void k_delz_from_zh(KARGS, Geo G, const double *zn, const double *phis, double *delz)
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
// the three cells at a cube vertex) of pfull and phi at the layer's two
// interfaces and of delp, staged through LDS, then the finite-volume
// pressure gradient along each D-grid edge.  Block: NPX x NPY corners; 33
// wide so that the n + 1 corner columns of C192 take 6 tiles (32 wide took 7,
// the last with one column), 7 rows so that its faces fit 256 threads.
// ====================================================================
#ifndef FV3_NHP_TX
#define FV3_NHP_TX 33
#endif
#ifndef FV3_NHP_TY
#define FV3_NHP_TY 7
#endif
constexpr int NPX = FV3_NHP_TX, NPY = FV3_NHP_TY;   // nh_p_grad corner tile
constexpr int NCW = NPX + 5, NCH = NPY + 5;   // cells i0-2..i0+NPX+2, j0-2..j0+NPY+2

// cell means x0..x3 of the cells m-2 .. m+1 to interface m: (-1,7,7,-1)/12,
// or with `edge` next to a tile edge (interfaces 0, n) the interface value
// of the quadratic with the three nearest cell means on the own side
// (1/3, 5/6, -1/6), on the edge the mean of the two sides' linear
// extrapolations (option edge_interp)
DEVI double face_mean(double x0, double x1, double x2, double x3, int m, int n, bool edge, const double *w4)
{
    if (edge) {
        if (m == 0 || m == n) return 0.75 * (x1 + x2) - 0.25 * (x0 + x3);
        if (m == 1 || m == n + 1) return (2.0 * x1 + 5.0 * x2 - x3) / 6.0;
        if (m == -1 || m == n - 1) return (2.0 * x2 + 5.0 * x1 - x0) / 6.0;
    }
    double r = 0.0;
    r += w4[0] * x0;
    r += w4[1] * x1;
    r += w4[2] * x2;
    r += w4[3] * x3;
    return r;
}

// Each block walks NHK consecutive layers of its corner tile: the corner
// values of p and phi at the interface below one layer are those above the
// next, so they are kept (two alternating LDS slots) instead of being
// interpolated again, and per layer only p, phi at the lower interface and
// delp are staged.  The next layer's cells and winds are loaded while the
// current layer computes.
#ifndef FV3_NHK
#define FV3_NHK 8
#endif
constexpr int NHK = FV3_NHK;
constexpr int NCS = (NCH * NCW + 255) / 256;    // staged cells per thread
constexpr int NBC = (NPY + 1) * (NPX + 1);      // corners of a block
constexpr int NPP = (NPX * NPY + 255) / 256;    // faces per thread
struct NhLds {
    double sc[3][NCH * NCW];   // staged cells (x-sweep view), then the x pass in place
    double sb[5][NBC];         // corner values: p, p (alternating interfaces), phi, phi, delp
};

// cells of the block's staging window into registers: p and phi of one
// interface and (WD) delp of one layer
template <class B, bool CORNER, bool WD>
DEVI void nh_load(const Geo &G, int i0, int j0, const double *Fp, const double *Fz, const B *D, double (&r)[NCS][3])
{
    const int n = G.n;
#pragma unroll
    for (int m = 0; m < NCS; m++) {
        const int e = (int)threadIdx.x + m * 256, rr = e / NCW, c = e - rr * NCW;
        const int i = i0 - 2 + c, j = j0 - 2 + rr;
        double a = 0.0, b = 0.0, d = 0.0;
        if (e < NCH * NCW && i <= n + 2 && j <= n + 2) {
            if constexpr (CORNER) {
                a = sv(G, Fp, SC, i, j, 0);
                b = sv(G, Fz, SC, i, j, 0);
                if constexpr (WD) d = (double)sv(G, D, SC, i, j, 0);
            } else {
                a = AT(Fp, i, j);
                b = AT(Fz, i, j);
                if constexpr (WD) d = (double)AT(D, i, j);
            }
        }
        r[m][0] = a;
        r[m][1] = b;
        r[m][2] = d;
    }
}

template <int NF>
DEVI void nh_store(NhLds &L, const double (&r)[NCS][3])
{
#pragma unroll
    for (int m = 0; m < NCS; m++) {
        const int e = (int)threadIdx.x + m * 256;
        if (e < NCH * NCW) {
#pragma unroll
            for (int f = 0; f < NF; f++) L.sc[f][e] = r[m][f];
        }
    }
}

// The tensor interpolation of the NF staged fields to the block's corners
// (into corner slots s0, s1, s2) in two passes: along x for every staged row
// at every corner column (into registers), then along y at each corner.
// Expects the staged cells to be visible (after a barrier); ends with one.
template <bool EI, bool CORNER, int NF>
DEVI void nh_corners(const Geo &G, int i0, int j0, NhLds &L, int s0, int s1, int s2, bool ebx, bool eby)
{
    const int n = G.n, tid = threadIdx.x;
    const int slot[3] = {s0, s1, s2};
    const double w4[4] = {-1.0 / 12.0, 7.0 / 12.0, 7.0 / 12.0, -1.0 / 12.0};
    constexpr int NRX = (NPY + 4) * (NPX + 1), NRP = (NRX + 255) / 256;
    double xr[NRP][NF];
#pragma unroll
    for (int m = 0; m < NRP; m++) {
        const int e = tid + m * 256, rr = e / (NPX + 1), c = e - rr * (NPX + 1);
        // the edge rule on rows inside the tile (row j = j0 - 2 + rr)
        const int jr = j0 - 2 + rr;
        const bool ex = EI && jr >= 0 && jr < n;
#pragma unroll
        for (int f = 0; f < NF; f++) {
            double rw = 0.0;
            if (e < NRX) {
                const double *row = &L.sc[f][rr * NCW + c];
                if (EI && ebx)
                    rw = face_mean(row[0], row[1], row[2], row[3], i0 + c, n, ex, w4);
                else
                    for (int a = 0; a < 4; a++) rw += w4[a] * row[a];
            }
            xr[m][f] = rw;
        }
    }
    // corners at cube vertices (corner blocks only): mean of the three
    // cells, from the staged cells
    if constexpr (CORNER) {
        for (int e = tid; e < NBC; e += 256) {
            const int r = e / (NPX + 1), c = e - r * (NPX + 1);
            const int i = i0 + c, j = j0 + r;
            if (i > n || j > n || !is_vertex(G, i, j)) continue;
            const int ci[4] = {i - 1, i, i, i - 1}, cj[4] = {j - 1, j - 1, j, j};
            for (int f = 0; f < NF; f++) {
                double sum = 0.0;
                for (int q = 0; q < 4; q++)
                    if (!in_corner(G, SC, ci[q], cj[q])) sum += L.sc[f][(cj[q] - j0 + 2) * NCW + (ci[q] - i0 + 2)];
                L.sb[slot[f]][e] = sum / 3.0;
            }
        }
    }
    __syncthreads();
    // the x pass in place of the staged cells (row rr, corner column c)
#pragma unroll
    for (int m = 0; m < NRP; m++) {
        const int e = tid + m * 256, rr = e / (NPX + 1), c = e - rr * (NPX + 1);
        if (e < NRX) {
#pragma unroll
            for (int f = 0; f < NF; f++) L.sc[f][rr * NCW + c] = xr[m][f];
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < (NBC + 255) / 256; m++) {
        const int e = tid + m * 256;
        if (e >= NBC) break;
        const int r = e / (NPX + 1), c = e - r * (NPX + 1);
        const int i = i0 + c, j = j0 + r;
        if (i > n || j > n || (CORNER && is_vertex(G, i, j))) continue;
#pragma unroll
        for (int f = 0; f < NF; f++) {
            double acc = 0.0;
            if (EI && eby) {
                const double *col = &L.sc[f][r * NCW + c];
                acc = face_mean(col[0], col[NCW], col[2 * NCW], col[3 * NCW], j, n, true, w4);
            } else {
                for (int b = 0; b < 4; b++) acc += w4[b] * L.sc[f][(r + b) * NCW + c];
            }
            L.sb[slot[f]][e] = acc;
        }
    }
    __syncthreads();
}

// CORNER: the block's staging window reaches a cube corner block, so its
// cell reads go through the corner views and its vertex corners take the
// three-cell mean; every other block reads the planes directly.
template <class B, bool EI, bool CORNER>
DEVI void nhpgrad_body(Bk bk, const Geo &G, const MetD &M, double bdt, const double *pfull, const double *phi,
                       const B *delp, B *u, B *v, NhLds &L)
{
    const int n = G.n, nz = G.nz, tid = threadIdx.x;
    const int i0 = bk.x * NPX, j0 = bk.y * NPY;
    const int nzb = (nz + NHK - 1) / NHK;
    const int t = (int)bk.z / nzb, k0 = ((int)bk.z % nzb) * NHK, k1 = k0 + NHK < nz ? k0 + NHK : nz;
    // with the edge rule, only blocks with corner columns (rows) within one
    // cell of a tile edge (0, 1, n - 1, n) take the one-sided branches of
    // the x (y) pass
    const bool ebx = EI && (i0 <= 1 || i0 + NPX >= n - 1), eby = EI && (j0 <= 1 || j0 + NPY >= n - 1);
    // edge lengths of the faces this thread updates (the same on every layer)
    double pdx[NPP], pdy[NPP];
#pragma unroll
    for (int m = 0; m < NPP; m++) {
        const int e = tid + m * 256, r = e / NPX, c = e - r * NPX;
        const int i = i0 + c, j = j0 + r;
        const bool in = e < NPX * NPY;
        pdx[m] = (in && i < n && j <= n) ? AT(MP(M, M_DX), i, j) : 1.0;
        pdy[m] = (in && i <= n && j < n) ? AT(MP(M, M_DY), i, j) : 1.0;
    }
    // the interface above the first layer
    double rg[NCS][3];
    nh_load<B, CORNER, false>(G, i0, j0, pfull + pidx(G, nz + 1, t, k0), phi + pidx(G, nz + 1, t, k0),
                              (const B *)nullptr, rg);
    nh_store<2>(L, rg);
    __syncthreads();
    nh_corners<EI, CORNER, 2>(G, i0, j0, L, 0, 2, 4, ebx, eby);
    nh_load<B, CORNER, true>(G, i0, j0, pfull + pidx(G, nz + 1, t, k0 + 1), phi + pidx(G, nz + 1, t, k0 + 1),
                             delp + pidx(G, nz, t, k0), rg);
    for (int k = k0; k < k1; k++) {
        const int b = 1 - ((k - k0) & 1), a = 1 - b;   // corner slots of the lower / upper interface
        const long o = pidx(G, nz, t, k);
        double pu[NPP], pv[NPP];
#pragma unroll
        for (int m = 0; m < NPP; m++) {
            const int e = tid + m * 256, r = e / NPX, c = e - r * NPX;
            const int i = i0 + c, j = j0 + r;
            const bool in = e < NPX * NPY;
            pu[m] = (in && i < n && j <= n) ? (double)AT(u + o, i, j) : 0.0;
            pv[m] = (in && i <= n && j < n) ? (double)AT(v + o, i, j) : 0.0;
        }
        nh_store<3>(L, rg);
        __syncthreads();
        if (k + 1 < k1)
            nh_load<B, CORNER, true>(G, i0, j0, pfull + pidx(G, nz + 1, t, k + 2), phi + pidx(G, nz + 1, t, k + 2),
                                     delp + pidx(G, nz, t, k + 1), rg);
        nh_corners<EI, CORNER, 3>(G, i0, j0, L, b, 2 + b, 4, ebx, eby);
        const double *P0 = L.sb[a], *P1 = L.sb[b], *Z0 = L.sb[2 + a], *Z1 = L.sb[2 + b], *DD = L.sb[4];
        // Each block owns the faces of its NPX x NPY corner rows/columns: the
        // grid spans corners 0..n, so a face row or column on a block boundary
        // is updated by exactly one block.  u on y-faces (i, j) uses corners
        // (i, j) and (i + 1, j); v on x-faces (i, j) corners (i, j) and (i, j + 1).
#pragma unroll
        for (int m = 0; m < NPP; m++) {
            const int e = tid + m * 256;
            if (e >= NPX * NPY) break;
            const int r = e / NPX, c = e - r * NPX;
            const int i = i0 + c, j = j0 + r;
            const int W = r * (NPX + 1) + c;
            if (i < n && j <= n) {
                const int E = W + 1;
                AT(u + o, i, j) = (B)pu[m] + (B)pgf(bdt, pdx[m], DD[W], DD[E], Z0[W], Z1[W], Z0[E], Z1[E], P0[W],
                                                    P1[W], P0[E], P1[E]);
            }
            if (i <= n && j < n) {
                const int E = W + (NPX + 1);
                AT(v + o, i, j) = (B)pv[m] + (B)pgf(bdt, pdy[m], DD[W], DD[E], Z0[W], Z1[W], Z0[E], Z1[E], P0[W],
                                                    P1[W], P0[E], P1[E]);
            }
        }
    }
}

template <class B, bool EI = false>
DEVI void k_nhpgrad(Bk bk, Geo G, MetD M, double bdt, const double *pfull, const double *phi, const B *delp, B *u,
                    B *v)
{
    __shared__ NhLds L;
    const int i0 = bk.x * NPX, j0 = bk.y * NPY;
    const bool corner = G.cube && (i0 - 2 < 0 || i0 + NPX + 2 >= G.n) && (j0 - 2 < 0 || j0 + NPY + 2 >= G.n);
    if (corner) nhpgrad_body<B, EI, true>(bk, G, M, bdt, pfull, phi, delp, u, v, L);
    else nhpgrad_body<B, EI, false>(bk, G, M, bdt, pfull, phi, delp, u, v, L);
}

// FP32 nh_p_grad compiled for six wavefronts per SIMD (its LDS allows six,
// its natural 95 VGPRs five; 75 VGPRs without spills)
#ifndef FV3_NHP_OCC
#define FV3_NHP_OCC 6
#endif
template <> constexpr int kocc<k_nhpgrad<float, false>> = FV3_NHP_OCC;

// ====================================================================
// utilities: fills, copies, finiteness check, tracer helpers, reductions
// ====================================================================
template <class T>
DEVI void k_fill(Bk bk, T *p, long count, T val)
{
    long e = (long)bk.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = val;
}
template <class TS, class TD>
DEVI void k_copy(Bk bk, const TS *s, TD *d, long count)
{
    long e = (long)bk.x * blockDim.x + threadIdx.x;
    if (e < count) d[e] = (TD)s[e];
}
template <class T>
static void fill(T *p, long count, T val, hipStream_t st)
{
    launch_fn<k_fill<T>>("k_fill", dim3((unsigned)((count + 255) / 256)), dim3(256), st, p, count, val);
}
template <class TS, class TD>
static void copy(const TS *s, TD *d, long count, hipStream_t st)
{
    launch_fn<k_copy<TS, TD>>("k_copy", dim3((unsigned)((count + 255) / 256)), dim3(256), st, s, d, count);
}

template <class T>
DEVI void k_check_finite(KARGS, Geo G, int L, const T *f, int *flags)
{
    KBEGIN(L);
    if (!isfinite((double)AT(f + pidx(G, L, t, k), i, j))) atomicOr(flags + 1, 1);
}

// tracer: area fluxes from the accumulated Courant numbers, scaled by 1/nsplt
template <class B>
DEVI void k_tracer_flux(KARGS, Geo G, MetD M, double rs, const B *cx, const B *cy,
                              const double *mfx, const double *mfy, B *crs, B *crys, B *xfx,
                              B *yfx, double *mxs, double *mys)
{
    KBEGIN(G.nz);
    int n = G.n;
    long o = pidx(G, G.nz, t, k);
    const double *dxa = MP(M, M_DXA), *dya = MP(M, M_DYA);
    if (i >= 0 && i <= n && j >= -3 && j <= n + 2) {
        double c = (double)AT(cx + o, i, j);
        int up = c > 0 ? i - 1 : i;
        AT(xfx + o, i, j) = (B)(c * pvx(G, dxa, dya, SC, up, j, 0, false) * AT(MP(M, M_DY), i, j) *
                                AT(MP(M, M_SIN_U), i, j) / rs);
        AT(crs + o, i, j) = (B)(c / rs);
        AT(mxs + o, i, j) = AT(mfx + o, i, j) / rs;
    }
    if (i >= -3 && i <= n + 2 && j >= 0 && j <= n) {
        double c = (double)AT(cy + o, i, j);
        int up = c > 0 ? j - 1 : j;
        AT(yfx + o, i, j) = (B)(c * pvy(G, dxa, dya, SC, i, up, 1, false) * AT(MP(M, M_DX), i, j) *
                                AT(MP(M, M_SIN_V), i, j) / rs);
        AT(crys + o, i, j) = (B)(c / rs);
        AT(mys + o, i, j) = AT(mfy + o, i, j) / rs;
    }
}

DEVI void k_tracer_dp(KARGS, Geo G, MetD M, const double *dp1, const double *mxs,
                            const double *mys, double *dp2)
{
    KBEGIN(G.nz);
    long o = pidx(G, G.nz, t, k);
    AT(dp2 + o, i, j) = AT(dp1 + o, i, j) + (AT(mxs + o, i, j) - AT(mxs + o, i + 1, j) + AT(mys + o, i, j) -
                                             AT(mys + o, i, j + 1)) /
                                                AT(MP(M, M_AREA), i, j);
}

// maximum that keeps a NaN (fmax drops it), so a non-finite Courant number
// reaches the host's sub-cycle count
DEVI double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }

// max |cx|, |cy| over the interior faces: block maximum, one atomic per block
template <class B>
__global__ void k_absmax(int ilo, int ihi, int jlo, int jhi, Geo G, const B *cx, const B *cy, unsigned long long *out)
{
    // each block covers its (i, j) patch on every gridDim.z-th plane, so that
    // only a few thousand blocks meet at the one atomic
    __shared__ double sm[256];
    int tid = threadIdx.y * blockDim.x + threadIdx.x;
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    double m = 0.0;
    if (i <= ihi && j <= jhi) {
        int n = G.n, planes = G.T * G.nz;
        for (int z = (int)blockIdx.z; z < planes; z += (int)gridDim.z) {
            int t = z / G.nz, k = z % G.nz;
            long o = pidx(G, G.nz, t, k);
            if (j < n) m = nanmax(m, fabs((double)AT(cx + o, i, j)));
            if (i < n) m = nanmax(m, fabs((double)AT(cy + o, i, j)));
        }
    }
    sm[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sm[tid] = nanmax(sm[tid], sm[tid + w]);
        __syncthreads();
    }
    // non-negative doubles order like their bit patterns, and a NaN's bits
    // lie above those of +inf, so a NaN survives the atomic too
    if (tid == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sm[0]));
}

// Neumaier-compensated sums: each thread sums its column over levels in a
// fixed order, then the block combines pairs (s, c) with Neumaier additions,
// one partial per block; the host adds the partials in order.
DEVI void neu_add(double &s, double &c, double x)
{
    double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

template <class B>
__global__ void k_mass_partial(int ilo, int ihi, int jlo, int jhi, Geo G, MetD M, const B *delp, const B *pt, const B *q,
                               int which, double *part)
{
    __shared__ double ss[256], sc[256];
    int tid = threadIdx.y * blockDim.x + threadIdx.x;
    int i = ilo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int j = jlo + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    int t = blockIdx.z;
    double s = 0.0, c = 0.0;
    if (i <= ihi && j <= jhi) {
        double ar = AT(MP(M, M_AREA), i, j);
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
template <class B>
struct Work {
    // bulk layer fields
    B *ax, *ay, *delpc, *ptc, *wc, *ke;
    B *ut, *vt, *crx, *cry, *xfx, *yfx, *FX, *FY, *VX, *VY, *dn, *pn, *wn, *om, *qo;
    // FP64 fields
    double *delzc, *s1, *s2, *s3, *dp1, *dp2, *mxs, *mys;
    double *pkc, *gz, *zh, *zn;   // interfaces
    unsigned long long *umax;
    double *part;
};

static long part_count(const fv3_grid *g)
{
    long bx = (g->n + 63) / 64, by = (g->n + 3) / 4;
    return bx * by * g->T;
}

template <class B>
static size_t carve(const fv3_grid *g, char *base, Work<B> *w)
{
    long el = alloc_elems(g, g->nz), ei = alloc_elems(g, g->nz + 1);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + 255) & ~(size_t)255;
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    B **bulk[] = {&w->ax, &w->ay, &w->delpc, &w->ptc, &w->wc, &w->ke, &w->ut, &w->vt, &w->crx, &w->cry,
                  &w->xfx, &w->yfx, &w->FX, &w->FY, &w->VX, &w->VY, &w->dn, &w->pn, &w->wn, &w->om, &w->qo};
    for (auto p : bulk) *p = (B *)take(el * sizeof(B));
    double **f64[] = {&w->delzc, &w->s1, &w->s2, &w->s3, &w->dp1, &w->dp2, &w->mxs, &w->mys};
    for (auto p : f64) *p = (double *)take(el * sizeof(double));
    double **f64i[] = {&w->pkc, &w->gz, &w->zh, &w->zn};
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
    if (g->bulk_bytes == 4) {
        Work<float> w;
        return carve(g, nullptr, &w);
    }
    Work<double> w;
    return carve(g, nullptr, &w);
}

template <class B>
static Mets<B> metrics_b(const fv3_grid *g);
template <>
Mets<double> metrics_b<double>(const fv3_grid *g)
{
    Mets<double> M;
    for (int m = 0; m < M_ALL; m++) M.m[m] = g->met[m];
    return M;
}
template <>
Mets<float> metrics_b<float>(const fv3_grid *g)
{
    Mets<float> M;
    for (int m = 0; m < M_ALL; m++) M.m[m] = g->metf[m];
    return M;
}
static MetD metrics_d(const fv3_grid *g) { return metrics_b<double>(g); }

// ====================================================================
// Host orchestration of one call
// ====================================================================
// The first column-solve pass in the instantiation the grid's options ask
// for: off-centring (beta < 1) and the cubic interface perturbation.
template <class F>
static void sim1_pass1(const fv3_grid *g, bool moist, F &&launch)
{
    using T_ = std::true_type;
    using F_ = std::false_type;
    using P2 = std::integral_constant<int, 2>;
    using P4 = std::integral_constant<int, 4>;
    const bool offc = g->p.beta != 1.0, cubic = g->p.pp_order == 4;
    auto go = [&](auto m) {
        if (offc && cubic) launch(T_{}, P4{}, m);
        else if (offc) launch(T_{}, P2{}, m);
        else if (cubic) launch(F_{}, P4{}, m);
        else launch(F_{}, P2{}, m);
    };
    if (moist) go(T_{});
    else go(F_{});
}

// the third column-solve pass: off-centring and humidity
template <class F>
static void sim1_pass3(const fv3_grid *g, bool moist, F &&launch)
{
    using T_ = std::true_type;
    using F_ = std::false_type;
    const bool offc = g->p.beta != 1.0;
    if (offc && moist) launch(T_{}, T_{});
    else if (offc) launch(T_{}, F_{});
    else if (moist) launch(F_{}, T_{});
    else launch(F_{}, F_{});
}

template <class B>
static fv3_status substeps_t(fv3_state *s, const fv3_grid *g, double dt, int n_split, int stop_stage,
                             hipStream_t st)
{
    Work<B> W;
    carve(g, (char *)s->workspace, &W);
    Mets<B> M = metrics_b<B>(g);
    MetD Md = metrics_d(g);
    const Geo &G = g->geo;
    int n = g->n, nz = g->nz, T = g->T, P = T * nz;
    long el = alloc_elems(g, nz);
    B *u = (B *)s->u, *v = (B *)s->v, *w = (B *)s->w, *delp = (B *)s->delp, *pt = (B *)s->pt;
    B *uc = (B *)s->uc, *vc = (B *)s->vc, *cx = (B *)s->cx, *cy = (B *)s->cy;
    double *delz = s->delz;
    const double *phis = s->phis;
    double bdt = dt / n_split, dt2 = 0.5 * bdt;
    const B *areaB = M.m[M_AREA];
    const B *qvp = (const B *)s->qv;
    const bool efix = g->p.edge_fix && g->edge_count > 0;

    // humidity is constant over the call: its halo once
    if (qvp) halo_set<B>(g, FieldSet<B>{{(B *)s->qv, nullptr, nullptr, nullptr}}, 1, nz, st);
    fill(s->mfx, el, 0.0, st);
    fill(s->mfy, el, 0.0, st);
    fill(cx, el, (B)0, st);
    fill(cy, el, (B)0, st);
    copy(delp, s->dp0, el, st);
    rec_mark();

    for (int it = 0; it < n_split; it++) {
        bool last = it == n_split - 1;
#define STOP(x) if (last && stop_stage == (x)) goto done
        // H-A
        halo_pair(g, g->planD, u, v, nz, st);
        if constexpr (std::is_same<B, double>::value) {
            halo_set<double>(g, FieldSet<double>{{delp, pt, w, delz}}, 4, nz, st);
        } else {
            halo_set<B>(g, FieldSet<B>{{delp, pt, w, nullptr}}, 3, nz, st);
            halo_scalar(g, delz, nz, st);
        }
        STOP(1);
        // c_sw
        {
            const dim3 cgrd((unsigned)((n + 3 + CTX - 1) / CTX), (unsigned)((n + 3 + CswRows<B>::Y - 1) / CswRows<B>::Y),
                            (unsigned)(T * ((nz + CSL - 1) / CSL)));
            if (g->p.edge_interp && g->p.kind == FV3_GRID_CUBED_SPHERE)
                launch_fn<k_csw<B, true>>("k_csw", cgrd, dim3(CNT), st, G, M, (B)dt2, (const B *)u, (const B *)v,
                                          (const B *)delp, (const B *)pt, (const B *)w, uc, vc, W.delpc, W.ptc,
                                          W.wc, W.ax, W.ay);
            else
                launch_fn<k_csw<B>>("k_csw", cgrd, dim3(CNT), st, G, M, (B)dt2, (const B *)u, (const B *)v,
                                    (const B *)delp, (const B *)pt, (const B *)w, uc, vc, W.delpc, W.ptc, W.wc,
                                    W.ax, W.ay);
        }
        STOP(2);
        // dz_c + riem_solver_c on the half-step cells
        launch_fn<k_dzc<B>>("k_dzc<B>", dim3((unsigned)sim1c_flat_blocks(n), 1, (unsigned)T), dim3(256), st, 0, -1, n,
                            -1, n, G, Md, (const double *)delz, phis, (const B *)W.ax, (const B *)W.ay, W.delzc);
        const dim3 fgrd((unsigned)sim1c_flat_blocks(n), 1, (unsigned)T);
        sim1_pass1(g, qvp != nullptr, [&](auto offc, auto ppo, auto moist) {
            launch_fn<k_sim1<B, B, 1, 0, decltype(offc)::value, decltype(ppo)::value, decltype(moist)::value>>(
                "k_sim1_c.p1", fgrd, dim3(256), st, 0, -1, n, -1, n, G, dt2, g->p.beta, g->p.ptop, (const B *)W.delpc,
                (const B *)W.ptc, qvp, (const double *)W.delzc, (const B *)W.wc, phis, W.s1, W.s2, W.s3, (B *)nullptr,
                (double *)nullptr, W.pkc, W.gz, 1);
        });
        launch2d_sh<k_sim1<B, B, 2, 0>>("k_sim1_c.p2", Shape{128, 2}, -1, n, -1, n, T, st, G, dt2, g->p.beta, g->p.ptop, (const B *)W.delpc,
                       (const B *)W.ptc, qvp, (const double *)W.delzc, (const B *)W.wc, phis, W.s1, W.s2, W.s3,
                       (B *)nullptr, (double *)nullptr, W.pkc, W.gz, 1);
        sim1_pass3(g, qvp != nullptr, [&](auto offc, auto moist) {
            launch_fn<k_sim1<B, B, 3, 0, decltype(offc)::value, 2, decltype(moist)::value>>(
                "k_sim1_c.p3", fgrd, dim3(256), st, 0, -1, n, -1, n, G, dt2, g->p.beta, g->p.ptop, (const B *)W.delpc,
                (const B *)W.ptc, qvp, (const double *)W.delzc, (const B *)W.wc, phis, W.s1, W.s2, W.s3, (B *)nullptr,
                (double *)nullptr, W.pkc, W.gz, 1);
        });
        launch2d_sh<k_sim1<B, B, 4, 0>>("k_sim1_c.p4", Shape{128, 2}, -1, n, -1, n, T, st, G, dt2, g->p.beta, g->p.ptop, (const B *)W.delpc,
                       (const B *)W.ptc, qvp, (const double *)W.delzc, (const B *)W.wc, phis, W.s1, W.s2, W.s3,
                       (B *)nullptr, (double *)nullptr, W.pkc, W.gz, 1);
        STOP(3);
        launch2d_s(k_pgradc<B>, (Shape{32, 8}), 0, n, 0, n, T * ((nz + PGK - 1) / PGK), st, G, Md, dt2, (const B *)W.delpc, (const double *)W.pkc,
                 (const double *)W.gz, uc, vc);
        STOP(4);
        halo_pair(g, g->planCv, uc, vc, nz, st);
        STOP(5);
        // d_sw
        launch2d_s(k_dsw_courant<B>, (Shape{16, 16}), -3, n + 2, -3, n + 2, P, st, G, M, (B)bdt, (const B *)uc, (const B *)vc, W.ut,
                 W.vt, W.crx, W.cry, W.xfx, W.yfx, g->flags);
        {
            FvArgs<B, B, B> a{};
            a.q = delp; a.Lq = nz; a.crx = W.crx; a.cry = W.cry; a.xfx = W.xfx; a.yfx = W.yfx;
            a.Lc = nz; a.area = areaB; a.epi = EPI_DELP; a.FX = W.FX; a.FY = W.FY; a.qout = W.dn;
            a.mfx = s->mfx; a.mfy = s->mfy; a.cxa = cx; a.cya = cy;
            fvtp(g, P, a, st);
            FvArgs<B, B, B> b{};
            b.q = pt; b.Lq = nz; b.crx = W.crx; b.cry = W.cry; b.xfx = W.xfx; b.yfx = W.yfx; b.Lc = nz;
            b.mx = W.FX; b.my = W.FY; b.area = areaB; b.epi = EPI_MASSW; b.qout = W.pn; b.dold = delp; b.dnew = W.dn;
            // edge-flux fix-up: keep the content fluxes (the C-grid half-step
            // arrays are free after p_grad_c)
            if (efix) { b.FX = W.delpc; b.FY = W.ptc; b.edges_only = 1; }
            fvtp(g, P, b, st);
            b.q = w; b.qout = W.wn;
            if (efix) { b.FX = W.wc; b.FY = W.qo; }
            fvtp(g, P, b, st);
        }
        // higher-order divergence damping (nord 1, 2): the C-grid half-step
        // arrays ax, ay are free after p_grad_c and hold the corner fields
        const B *hd = nullptr;
        double hc = 0.0;
        if (g->p.nord > 0 && g->p.d4_bg > 0.0) {
            launch2d(k_cdiv<B>, 0, n, 0, n, P, st, G, M, (const B *)u, (const B *)v, W.ax);
            B *a = W.ax, *b = W.ay;
            for (int r = 0; r < g->p.nord; r++) {
                halo_corner(g, a, nz, st);
                launch2d(k_clap<B>, 0, n, 0, n, P, st, G, M, (const B *)a, b);
                std::swap(a, b);
            }
            hd = a;
            hc = (g->p.nord % 2 ? 1.0 : -1.0) * std::pow(g->p.d4_bg * g->da_min, g->p.nord + 1);
        }
        const bool eppm = g->p.edge_ppm && g->p.kind == FV3_GRID_CUBED_SPHERE;
        auto omke = [&](auto lim) {
            if constexpr (sizeof(B) == 4)
                launch_fn<k_dsw_omke<B, decltype(lim)::value>>(
                    "k_dsw_omke<B>", dim3((unsigned)(((n + 6) * (n + 6) + 255) / 256), 1, (unsigned)P), dim3(256), st,
                    0, -3, n + 2, -3, n + 2, G, M, (B)bdt, (B)g->p.d2_bg, (B)(g->p.dddmp * bdt), (B)g->da_min,
                    (const B *)u, (const B *)v, (const B *)W.ut, (const B *)W.vt, (const B *)hd, (B)hc, W.om, W.ke);
            else
                launch2d_sh<k_dsw_omke<B, decltype(lim)::value>>(
                    "k_dsw_omke<B>", Shape{16, 16}, -3, n + 2, -3, n + 2, P, st, G, M, (B)bdt, (B)g->p.d2_bg,
                    (B)(g->p.dddmp * bdt), (B)g->da_min, (const B *)u, (const B *)v, (const B *)W.ut,
                    (const B *)W.vt, (const B *)hd, (B)hc, W.om, W.ke);
        };
        if (g->p.hord == 6) omke(std::integral_constant<int, 6>{});
        else if (g->p.hord == 5) omke(std::integral_constant<int, 5>{});
        else omke(std::integral_constant<int, 8>{});
        if (eppm) {
            const int cnt = 12 * (n + 1) - 36;
            auto kee = [&](auto lim) {
                launch_fn<k_ke_edge<B, decltype(lim)::value>>("k_ke_edge", dim3((cnt + 255) / 256, nz, 6), dim3(256),
                                                             st, G, M, (B)bdt, (const B *)u, (const B *)v,
                                                             (const B *)W.ut, (const B *)W.vt, W.ke);
            };
            if (g->p.hord == 6) kee(std::integral_constant<int, 6>{});
            else if (g->p.hord == 5) kee(std::integral_constant<int, 5>{});
            else kee(std::integral_constant<int, 8>{});
        }
        {
            FvArgs<B, B, B> a{};
            a.q = W.om; a.Lq = nz; a.crx = W.crx; a.cry = W.cry; a.xfx = W.xfx; a.yfx = W.yfx; a.Lc = nz;
            a.area = areaB; a.epi = EPI_FLUX; a.FX = W.VX; a.FY = W.VY;
            fvtp(g, P, a, st);
        }
        launch2d_s(k_dsw_update<B>, (Shape{32, 8}), 0, n, 0, n, P, st, G, M, (const B *)W.ke, (const B *)W.VX, (const B *)W.VY,
                 (const B *)W.dn, (const B *)W.pn, (const B *)W.wn, (const B *)W.om, (B)(g->p.vtdm * g->da_min), u, v,
                 delp, pt, w);
        if (efix)
            launch_fn<k_edgefix_dsw<B>>("k_edgefix", dim3((g->edge_count + 255) / 256, nz), dim3(256), st, G,
                                        (const EdgeCell *)g->edge_cells, g->edge_count, areaB, (const B *)W.FX,
                                        (const B *)W.FY, (const B *)W.delpc, (const B *)W.ptc, (const B *)W.wc,
                                        (const B *)W.qo, delp, pt, w, s->mfx, s->mfy);
        STOP(6);
        // dz_d
        if constexpr (std::is_same<B, float>::value) {
            // FP32 deviations from per-interface reference heights: the input
            // and the references in the FP64 height scratch zh (the input
            // fills half of it), the output in zn
            const long ei = alloc_elems(g, nz + 1);
            float *zd = (float *)W.zh, *zdn = (float *)W.zn;
            double *zref = (double *)((float *)W.zh + ((ei + 63) / 64) * 64);
            launch2d(k_heights_dev, -3, n + 2, -3, n + 2, T, st, G, (const double *)delz, phis, zref, zd);
            FvArgs<float, B, double> a{};
            a.q = zd; a.Lq = nz + 1; a.crx = W.crx; a.cry = W.cry; a.xfx = W.xfx; a.yfx = W.yfx; a.Lc = nz;
            a.iface = 1; a.area = M.m[M_AREA]; a.epi = EPI_ADV; a.qout = zdn;
            fvtp(g, P, a, st);
            launch2d(k_delz_from_zdev, 0, n - 1, 0, n - 1, P, st, G, (const float *)zdn, (const double *)zref, phis,
                     delz);
        } else {
            launch2d(k_heights, -3, n + 2, -3, n + 2, T, st, G, (const double *)delz, phis, W.zh);
            FvArgs<double, B, double> a{};
            a.q = W.zh; a.Lq = nz + 1; a.crx = W.crx; a.cry = W.cry; a.xfx = W.xfx; a.yfx = W.yfx; a.Lc = nz;
            a.iface = 1; a.area = Md.m[M_AREA]; a.epi = EPI_ADV; a.qout = W.zn;
            fvtp(g, P, a, st);
            launch2d(k_delz_from_zh, 0, n - 1, 0, n - 1, P, st, G, (const double *)W.zn, phis, delz);
        }
        STOP(7);
        // riem_solver3
        sim1_pass1(g, qvp != nullptr, [&](auto offc, auto ppo, auto moist) {
            launch2d_fn<k_sim1<B, B, 1, 1, decltype(offc)::value, decltype(ppo)::value, decltype(moist)::value>>(
                "k_sim1_3.p1", 0, n - 1, 0, n - 1, T, st, G, bdt, g->p.beta, g->p.ptop, (const B *)delp,
                (const B *)pt, qvp, (const double *)delz, (const B *)w, phis, W.s1, W.s2, W.s3, w, delz, s->pfull,
                s->phi, 0);
        });
        launch2d_fn<k_sim1<B, B, 2, 1>>("k_sim1_3.p2", 0, n - 1, 0, n - 1, T, st, G, bdt, g->p.beta, g->p.ptop, (const B *)delp,
                       (const B *)pt, qvp, (const double *)delz, (const B *)w, phis, W.s1, W.s2, W.s3, w, delz,
                       s->pfull, s->phi, 0);
        sim1_pass3(g, qvp != nullptr, [&](auto offc, auto moist) {
            launch2d_fn<k_sim1<B, B, 3, 1, decltype(offc)::value, 2, decltype(moist)::value>>(
                "k_sim1_3.p3", 0, n - 1, 0, n - 1, T, st, G, bdt, g->p.beta, g->p.ptop, (const B *)delp,
                (const B *)pt, qvp, (const double *)delz, (const B *)w, phis, W.s1, W.s2, W.s3, w, delz, s->pfull,
                s->phi, 0);
        });
        launch2d_fn<k_sim1<B, B, 4, 1>>("k_sim1_3.p4", 0, n - 1, 0, n - 1, T, st, G, bdt, g->p.beta, g->p.ptop, (const B *)delp,
                       (const B *)pt, qvp, (const double *)delz, (const B *)w, phis, W.s1, W.s2, W.s3, w, delz,
                       s->pfull, s->phi, 0);
        STOP(8);
        // H-C
        halo_set<double>(g, FieldSet<double>{{s->pfull, s->phi, nullptr, nullptr}}, 2, nz + 1, st);
        halo_scalar(g, delp, nz, st);
        STOP(9);
        // nh_p_grad
        {
            const dim3 ngrd((n + NPX) / NPX, (n + NPY) / NPY, T * ((nz + NHK - 1) / NHK));
            if (g->p.edge_interp && g->p.kind == FV3_GRID_CUBED_SPHERE)
                launch_fn<k_nhpgrad<B, true>>("k_nhpgrad", ngrd, dim3(256), st, G, Md, bdt, (const double *)s->pfull,
                                              (const double *)s->phi, (const B *)delp, u, v);
            else
                launch_fn<k_nhpgrad<B>>("k_nhpgrad", ngrd, dim3(256), st, G, Md, bdt, (const double *)s->pfull,
                                        (const double *)s->phi, (const B *)delp, u, v);
        }
#undef STOP
    }
    rec_mark();
done:
    {
        B *chk[] = {u, v, w, delp, pt};
        for (B *f : chk) launch2d(k_check_finite<B>, 0, n - 1, 0, n - 1, P, st, G, nz, (const B *)f, g->flags);
        launch2d(k_check_finite<double>, 0, n - 1, 0, n - 1, P, st, G, nz, (const double *)delz, g->flags);
    }
    if (hipGetLastError() != hipSuccess) return FV3_EDEVICE;
    return FV3_OK;
}

fv3_status record_substeps(fv3_state *s, const fv3_grid *g, double bdt, Recorder *rec)
{
    rec->pos = 0;
    rec->mark = 0;
    g_rec = rec;
    fv3_status r = g->bulk_bytes == 4 ? substeps_t<float>(s, g, bdt, 1, 0, nullptr)
                                      : substeps_t<double>(s, g, bdt, 1, 0, nullptr);
    g_rec = nullptr;
    if (r != FV3_OK) return r;
    // a member whose options choose other kernels than the first member's
    if (rec->bad || rec->pos != rec->sites.size() || rec->mark != 2) return FV3_EUNSUPPORTED;
    return FV3_OK;
}

fv3_status run_substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split, int stop_stage,
                        hipStream_t st)
{
    if (g->bulk_bytes == 4) return substeps_t<float>(s, g, dt, n_split, stop_stage, st);
    return substeps_t<double>(s, g, dt, n_split, stop_stage, st);
}

fv3_status run_halo_cells(const fv3_grid *g, void *const *f, int nf, int levels, int fp64,
                          hipStream_t st)
{
    for (int q = 0; q < nf; q++) {
        if (fp64 || g->bulk_bytes == 8) halo_scalar(g, (double *)f[q], levels, st);
        else halo_scalar(g, (float *)f[q], levels, st);
    }
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

fv3_status run_halo_pair_cells(const fv3_grid *g, void *fx, void *fy, int levels, int fp64,
                               hipStream_t st)
{
    if (fp64 || g->bulk_bytes == 8) halo_pair(g, g->planA, (double *)fx, (double *)fy, levels, st);
    else halo_pair(g, g->planA, (float *)fx, (float *)fy, levels, st);
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

template <class B>
static fv3_status tracer_t(void *const *q, int nq, fv3_state *s, const fv3_grid *g, int nsplt, hipStream_t st)
{
    Work<B> W;
    carve(g, (char *)s->workspace, &W);
    Mets<B> M = metrics_b<B>(g);
    MetD Md = metrics_d(g);
    const Geo &G = g->geo;
    int n = g->n, nz = g->nz, P = g->T * nz;
    long el = alloc_elems(g, nz);
    B *cx = (B *)s->cx, *cy = (B *)s->cy;
    halo_pair(g, g->planCv, cx, cy, nz, st);
    if (nsplt <= 0) {
        unsigned long long zero = 0, h = 0;
        fill(W.umax, 1, zero, st);
        launch2d_native("k_absmax", k_absmax<B>, 0, n, 0, n, P < 8 ? P : 8, st, G, (const B *)cx, (const B *)cy,
                        W.umax);
        if (hipMemcpyAsync(&h, W.umax, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return FV3_EDEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return FV3_EDEVICE;
        double cmax;
        std::memcpy(&cmax, &h, sizeof(cmax));
        if (!std::isfinite(cmax))
            return set_error(FV3_ENONFINITE, "accumulated Courant numbers cx, cy are not finite");
        if (cmax > (double)FV3_MAX_TRACER_SUBCYCLES)
            return set_error(FV3_ECFL, "max |cx|, |cy| = " + std::to_string(cmax) + " needs more than " +
                                           std::to_string(FV3_MAX_TRACER_SUBCYCLES) + " tracer sub-cycles");
        nsplt = (int)std::ceil(cmax);
        if (nsplt < 1) nsplt = 1;
    }
    double rs = (double)nsplt;
    const bool efix = g->p.edge_fix && g->edge_count > 0;
    launch2d_s(k_tracer_flux<B>, (Shape{128, 2}), -3, n + 3, -3, n + 3, P, st, G, Md, rs, (const B *)cx, (const B *)cy,
             (const double *)s->mfx, (const double *)s->mfy, W.crx, W.cry, W.xfx, W.yfx, W.mxs, W.mys);
    copy(s->dp0, W.dp1, el, st);
    double *dp1 = W.dp1, *dp2 = W.dp2;
    for (int itr = 0; itr < nsplt; itr++) {
        launch2d(k_tracer_dp, 0, n - 1, 0, n - 1, P, st, G, Md, (const double *)dp1, (const double *)W.mxs,
                 (const double *)W.mys, dp2);
        for (int m = 0; m < nq; m++) {
            B *Q = (B *)q[m];
            halo_scalar(g, Q, nz, st);
            FvArgs<B, B, double> a{};
            a.q = Q; a.Lq = nz; a.crx = W.crx; a.cry = W.cry; a.xfx = W.xfx; a.yfx = W.yfx; a.Lc = nz;
            a.mx = W.mxs; a.my = W.mys; a.area = M.m[M_AREA]; a.epi = EPI_TRACER; a.qout = W.qo;
            a.dp1 = dp1; a.dp2 = dp2;
            if (efix) { a.FX = W.delpc; a.FY = W.ptc; a.edges_only = 1; }
            fvtp(g, P, a, st);
            copy((const B *)W.qo, Q, el, st);
            if (efix)
                launch_fn<k_edgefix_q<B>>("k_edgefix_q", dim3((g->edge_count + 255) / 256, nz), dim3(256), st, G,
                                          (const EdgeCell *)g->edge_cells, g->edge_count, (const B *)M.m[M_AREA],
                                          (const B *)W.delpc, (const B *)W.ptc, (const double *)dp2, Q);
        }
        double *tmp = dp1;
        dp1 = dp2;
        dp2 = tmp;
    }
    for (int m = 0; m < nq; m++) halo_scalar(g, (B *)q[m], nz, st);   // leave consistent halos
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

fv3_status run_tracer(void *const *q, int nq, fv3_state *s, const fv3_grid *g, int nsplt,
                      hipStream_t st)
{
    if (g->bulk_bytes == 4) return tracer_t<float>(q, nq, s, g, nsplt, st);
    return tracer_t<double>(q, nq, s, g, nsplt, st);
}

template <class B>
static fv3_status mass_sums_t(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                              int nq, double *out, hipStream_t st)
{
    MetD M = metrics_d(g);
    const Geo &G = g->geo;
    int n = g->n;
    long np = part_count(g);
    double *part = g->red;
    std::vector<double> h(2 * np);
    for (int which = 0; which < 2 + nq; which++) {
        const B *qq = which >= 2 ? (const B *)q[which - 2] : nullptr;
        launch2d_native("k_mass_partial", k_mass_partial<B>, 0, n - 1, 0, n - 1, g->T, st, G, M, (const B *)delp, (const B *)pt, qq,
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

// Streaming copy for the bandwidth roof: 16-byte loads and stores; a block
// moves 16 KiB per iteration (four loads per thread issued before the four
// stores), grid-stride over 16 KiB chunks with at most 2048 blocks (8 per
// compute unit).
__global__ void __launch_bounds__(256) k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     long n16)
{
    const long stride = (long)gridDim.x * 1024;
    for (long base = (long)blockIdx.x * 1024; base < n16; base += stride) {
        uint4 r[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            long e = base + u * 256 + threadIdx.x;
            if (e < n16) r[u] = src[e];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            long e = base + u * 256 + threadIdx.x;
            if (e < n16) dst[e] = r[u];
        }
    }
}

fv3_status run_device_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    long n16 = (long)(bytes / 16);
    bool tm = timing_wanted("k_stream_copy");
    TimingRec r;
    if (tm) timing_begin("k_stream_copy", st, r);
    if (n16 > 0) {
        long chunks = (n16 + 1023) / 1024;
        unsigned blocks = (unsigned)(chunks < 2048 ? chunks : 2048);
        hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16);
    }
    if (tm) timing_end(st, r);
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

fv3_status run_mass_sums(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                         int nq, double *out, hipStream_t st)
{
    if (g->bulk_bytes == 4) return mass_sums_t<float>(g, delp, pt, q, nq, out, st);
    return mass_sums_t<double>(g, delp, pt, q, nq, out, st);
}

// ====================================================================
// Allocation-free mass sums.  The per-block partials go to a fixed
// file-scope device array instead of the grid's reduction buffer, and one
// thread combines them on the device into the caller's device output, so
// the call allocates nothing (device or host) and does not synchronise.
// Each GPU holds its own copy of the array; host code only ever uses the
// address that hipGetSymbolAddress returned for the current device.
// ====================================================================
static __device__ __align__(256) double scratch[FV3_NOALLOC_SCRATCH_BYTES / sizeof(double)];

static std::mutex g_scratch_mu;
static double *g_scratch_dev[FV3_MAX_DEVICES];   // device address of `scratch`, per HIP ordinal

fv3_status noalloc_setup(int device)
{
    if (device < 0 || device >= FV3_MAX_DEVICES) return FV3_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return FV3_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FV3_EDEVICE;
    g_scratch_dev[device] = (double *)p;
    return FV3_OK;
}

long noalloc_mass_doubles(const fv3_grid *g) { return 2 * part_count(g); }

// The block partials added in block order with the same Neumaier steps as
// the host-side combine of run_mass_sums, so both give the same bits.
__global__ void k_mass_final(const double *part, long np, double *out)
{
    if (threadIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (long b = 0; b < np; b++) {
        c += part[2 * b + 1];
        double x = part[2 * b], t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    *out = s + c;
}

template <class B>
static fv3_status mass_sums_noalloc_t(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                                      int nq, double *dev_out, double *part, hipStream_t st)
{
    MetD M = metrics_d(g);
    const Geo &G = g->geo;
    int n = g->n;
    long np = part_count(g);
    // every block of k_mass_partial writes its own two slots (zero outside
    // the interior), so nothing in the scratch has to be cleared first
    for (int which = 0; which < 2 + nq; which++) {
        const B *qq = which >= 2 ? (const B *)q[which - 2] : nullptr;
        launch2d_native("k_mass_partial", k_mass_partial<B>, 0, n - 1, 0, n - 1, g->T, st, G, M, (const B *)delp,
                        (const B *)pt, qq, which < 2 ? which : 2, part);
        hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(64), 0, st, (const double *)part, np, dev_out + which);
    }
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

fv3_status run_mass_sums_noalloc(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                                 int nq, double *dev_out, hipStream_t st)
{
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (g->p.device >= 0 && g->p.device < FV3_MAX_DEVICES) part = g_scratch_dev[g->p.device];
    }
    if (!part) return FV3_EINTERNAL;   // fv3_init_grid resolves it for the grid's device
    if (g->bulk_bytes == 4) return mass_sums_noalloc_t<float>(g, delp, pt, q, nq, dev_out, part, st);
    return mass_sums_noalloc_t<double>(g, delp, pt, q, nq, dev_out, part, st);
}

}  // namespace fv3
