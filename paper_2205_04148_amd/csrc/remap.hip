// Vertical remapping of the remapping step (Sec. II): the deformed Lagrangian
// layers of every column are mapped back to the reference interfaces
// pe_K = ak_K + bk_K ps (ps = ptop + the column's sum of delp) by a
// mass-conserving piecewise-parabolic remap in pressure.
//
// Reconstruction (Colella-Woodward PPM on non-uniform layers): interface
// values by fourth-order interpolation of the layer means with monotonised
// slopes where two layers lie on each side, thickness-weighted linear
// interpolation next to the top and bottom layers, constant top and bottom
// layers, and the monotonicity limiter on each parabola.  Fields: pt, w and
// the tracers as they are, delz as delz/delp (its remapped integral is the
// new delz, so the column depth is kept), the D-grid winds at faces on the
// mean interfaces of the two cells that share the face; delp becomes the
// reference thickness.
//
// GPU mapping: one thread per (column, field), 64 consecutive columns per
// wavefront so that every level load is one coalesced row segment.  A thread
// walks its column once, top to bottom, over the merged sequence of source
// and target interfaces, keeping a five-layer window of means and
// thicknesses in registers and the interface value below the current layer
// (which becomes the one above the next).  The walk finishes target layers
// before it has read every source layer they could overwrite, so results go
// to workspace slots and are copied back.  All arithmetic is FP64.
#include <cmath>
#include <string>

#include "fv3_internal.hpp"

namespace fv3 {
namespace {

constexpr int RMAX = FV3_REMAP_MAX_LEVELS;
constexpr int RSLOTS = 8;   // fields per launch, at most
constexpr int RNF = 4;      // cell fields per thread (one walk of the column serves them all)
enum { RM_CELL = 0, RM_U = 1, RM_V = 2 };

// reference coordinate, passed by value in the kernel arguments
struct RCoef {
    double ak[RMAX + 1], bk[RMAX + 1];
};

struct RBatch {
    const void *src[RSLOTS];
    void *dst[RSLOTS];
    int fp64[RSLOTS];    // 1: the field is FP64, else bulk precision
    int ratio[RSLOTS];   // 1: remap field / delp, store its integral (delz)
    int nf;
};

__device__ __forceinline__ double ld(const void *p, long e, bool fp64, bool bulk64)
{
    if (fp64 || bulk64) return ((const double *)p)[e];
    return (double)((const float *)p)[e];
}

__device__ __forceinline__ void st(void *p, long e, bool fp64, bool bulk64, double v)
{
    if (fp64 || bulk64) ((double *)p)[e] = v;
    else ((float *)p)[e] = (float)v;
}

// monotonised slope from the raw slope and the two one-sided differences
__device__ __forceinline__ double mono(double raw, double lo, double hi)
{
    if (lo * hi <= 0.0) return 0.0;
    return copysign(fmin(fabs(raw), 2.0 * fmin(fabs(lo), fabs(hi))), raw);
}

// Remap up to NF fields of one column (cell or face, by MODE) in one walk.
// The layer geometry (reciprocals of the thickness sums of the interface
// interpolation, the layer's own reciprocal thickness) is computed once per
// source layer for all fields; the limited slope of layer s + 1, needed by the
// interface below layer s, is kept for the interface below layer s + 1.
template <int MODE, int NF>
__global__ __launch_bounds__(256) void k_remap(Geo G, int bulk64, double ptop, RCoef C, RBatch F,
                                               const void *delp, int *flags)
{
    const int n = G.n, nz = G.nz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    const int ni = MODE == RM_V ? n + 1 : n, nj = MODE == RM_U ? n + 1 : n;
    if (i >= ni || j >= nj) return;
    const int groups = (F.nf + NF - 1) / NF;
    const int t = (int)blockIdx.z / groups, f0 = ((int)blockIdx.z % groups) * NF;
    const int nfg = min(NF, F.nf - f0);
    const bool b64 = bulk64 != 0;
    const long lev = G.lev;
    const long c0 = G.off0 + (long)t * nz * lev + (long)j * G.pitch + i;
    const long c1 = MODE == RM_U ? c0 - G.pitch : MODE == RM_V ? c0 - 1 : c0;   // other cell of a face

    auto thick = [&](int k) -> double {
        long o = (long)k * lev;
        if (MODE == RM_CELL) return ld(delp, c0 + o, false, b64);
        return 0.5 * (ld(delp, c0 + o, false, b64) + ld(delp, c1 + o, false, b64));
    };
    // surface pressure, summed in the same order as the walk's interfaces
    double ps = ptop;
    for (int k = 0; k < nz; k++) ps += thick(k);

    // window over layers s-1 .. s+2 (positions 1..4): thicknesses d1..d4,
    // means a2..a4 per field (layer s-1 enters only through its slope and
    // thickness); b3, b4 = bottom interfaces of layers s+1, s+2 as summed
    double d1 = 1, d2 = 1, d3 = 1, d4 = 1, pa = ptop, b2 = ptop, b3 = ptop, b4 = ptop;
    double a2[NF], a3[NF], a4[NF];
    auto next = [&](int k, double *a, double &d, double &bot) {
        if (k >= nz) return;
        double h = thick(k), bb = pa + h;
        d = bb - pa;
        pa = bb;
        bot = bb;
        double rh = 1.0 / h;
#pragma unroll
        for (int q = 0; q < NF; q++) {
            if (q < nfg) {
                double v = ld(F.src[f0 + q], c0 + (long)k * lev, F.fp64[f0 + q] != 0, b64);
                a[q] = F.ratio[f0 + q] ? v * rh : v;
            }
        }
    };
#pragma unroll
    for (int q = 0; q < NF; q++) a2[q] = a3[q] = a4[q] = 0.0;
    next(0, a2, d2, b2);
    next(1, a3, d3, b3);
    next(2, a4, d4, b4);

    // limited slope of the layer at position 3 (layers s, s+1, s+2 at
    // positions 2, 3, 4) for every field
    double sl3[NF];
    auto slope3 = [&](bool have) {
        double r = 1.0 / (d2 + d3 + d4), kh = d3 * r * (2.0 * d2 + d3) / (d4 + d3),
               kl = d3 * r * (d3 + 2.0 * d4) / (d2 + d3);
#pragma unroll
        for (int q = 0; q < NF; q++) {
            double lo = a3[q] - a2[q], hi = a4[q] - a3[q];
            sl3[q] = have ? mono(kh * hi + kl * lo, lo, hi) : 0.0;
        }
    };
    slope3(nz >= 3);
    // interface values below layer s (K = s + 1) before limiting; sl2 = the
    // limited slope of layer s
    double eR[NF], l[NF], r[NF], c6[NF], acc[NF];
    auto below = [&](int s, const double *sl2) {
        const int K = s + 1;
        if (K >= 2 && K <= nz - 2) {
            double s23 = d2 + d3, rs = 1.0 / s23, rsum = 1.0 / (d1 + d2 + d3 + d4);
            double cj = d2 * rs;
            double w = 2.0 * d3 * d2 * rs * ((d1 + d2) / (2.0 * d2 + d3) - (d4 + d3) / (2.0 * d3 + d2));
            double g1 = d3 * (d3 + d4) / (d2 + 2.0 * d3), g2 = d2 * (d1 + d2) / (2.0 * d2 + d3);
#pragma unroll
            for (int q = 0; q < NF; q++) {
                double jump = a3[q] - a2[q];
                eR[q] = a2[q] + cj * jump + (w * jump - g2 * sl3[q] + g1 * sl2[q]) * rsum;
            }
        } else {
            double rs = 1.0 / (d2 + d3);
#pragma unroll
            for (int q = 0; q < NF; q++) eR[q] = (a2[q] * d3 + a3[q] * d2) * rs;
        }
    };
    {
        double zero[NF];
#pragma unroll
        for (int q = 0; q < NF; q++) {
            zero[q] = 0.0;
            eR[q] = a2[q];
        }
        if (nz > 1) below(0, zero);
    }
#pragma unroll
    for (int q = 0; q < NF; q++) {
        l[q] = r[q] = a2[q];   // layer 0 is constant
        c6[q] = 0.0;
        acc[q] = 0.0;
    }
    int s = 0;
    // both walks end on ps exactly
    double top1 = ptop, bot1 = nz > 1 ? b2 : ps, rds = 1.0 / (bot1 - top1);
    double top2 = ptop, bot2 = nz > 1 ? C.ak[1] + C.bk[1] * ps : ps;
    double cur = ptop;
    int m = 0;
    bool bad = false;
    for (int it = 0; it <= 2 * nz; it++) {
        double nxt = fmin(bot1, bot2);
        double x1 = (cur - top1) * rds, x2 = (nxt - top1) * rds;
        // integral over [x1, x2] of l + x (r - l + c6 (1 - x)), times the thickness
        double h = (nxt - cur), sx = 0.5 * (x1 + x2), qx = (x1 * x1 + x1 * x2 + x2 * x2) * (1.0 / 3.0);
#pragma unroll
        for (int q = 0; q < NF; q++) acc[q] += h * (l[q] + (r[q] - l[q] + c6[q]) * sx - c6[q] * qx);
        cur = nxt;
        if (nxt >= bot2) {   // target layer m complete
            double dm = bot2 - top2, rdm = 1.0 / dm;
            bad |= !(dm > 0.0);
#pragma unroll
            for (int q = 0; q < NF; q++) {
                if (q < nfg)
                    st(F.dst[f0 + q], c0 + (long)m * lev, F.fp64[f0 + q] != 0, b64,
                       F.ratio[f0 + q] ? acc[q] : acc[q] * rdm);
                acc[q] = 0.0;
            }
            top2 = bot2;
            if (++m == nz) break;
            bot2 = m + 1 < nz ? C.ak[m + 1] + C.bk[m + 1] * ps : ps;
        }
        if (nxt >= bot1 && s < nz - 1) {   // into source layer s + 1
            s++;
            double sl2[NF];
#pragma unroll
            for (int q = 0; q < NF; q++) {
                a2[q] = a3[q];
                a3[q] = a4[q];
                sl2[q] = sl3[q];
            }
            d1 = d2; d2 = d3; d3 = d4;
            top1 = bot1;
            bot1 = s < nz - 1 ? b3 : ps;
            rds = 1.0 / (bot1 - top1);
            b3 = b4;
            next(s + 2, a4, d4, b4);
            slope3(s + 2 <= nz - 1);
            double eL[NF];
#pragma unroll
            for (int q = 0; q < NF; q++) eL[q] = eR[q];
            if (s < nz - 1) below(s, sl2);
#pragma unroll
            for (int q = 0; q < NF; q++) {
                double lq = eL[q], rq = eR[q], aq = a2[q];
                if (s == nz - 1) {
                    lq = rq = aq;
                } else if ((rq - aq) * (aq - lq) <= 0.0) {
                    lq = rq = aq;
                } else {
                    double dq = rq - lq, cc = 6.0 * (aq - 0.5 * (lq + rq));
                    if (dq * cc > dq * dq) lq = 3.0 * aq - 2.0 * rq;
                    else if (-dq * dq > dq * cc) rq = 3.0 * aq - 2.0 * lq;
                }
                l[q] = lq;
                r[q] = rq;
                c6[q] = 6.0 * (aq - 0.5 * (lq + rq));
            }
        }
    }
    if (bad || m != nz) atomicOr(flags + 2, 1);
}

// copy the remapped interior points of the batch back into the fields
template <int MODE>
__global__ __launch_bounds__(256) void k_remap_back(Geo G, int bulk64, RBatch F)
{
    const int n = G.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    const int ni = MODE == RM_V ? n + 1 : n, nj = MODE == RM_U ? n + 1 : n;
    if (i >= ni || j >= nj) return;
    const int z = (int)blockIdx.z, f = z % F.nf, tk = z / F.nf;   // tk = t * nz + k
    const long e = G.off0 + (long)tk * G.lev + (long)j * G.pitch + i;
    const bool b64 = bulk64 != 0, f64 = F.fp64[f] != 0;
    st((void *)F.src[f], e, f64, b64, ld(F.dst[f], e, f64, b64));
}

// delp of every column becomes the reference thickness
__global__ __launch_bounds__(256) void k_remap_delp(Geo G, int bulk64, double ptop, RCoef C, void *delp)
{
    const int n = G.n, nz = G.nz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const bool b64 = bulk64 != 0;
    const long c0 = G.off0 + (long)blockIdx.z * nz * G.lev + (long)j * G.pitch + i;
    double ps = ptop;
    for (int k = 0; k < nz; k++) ps += ld(delp, c0 + (long)k * G.lev, false, b64);
    double top = ptop;
    for (int k = 0; k < nz; k++) {
        double bot = C.ak[k + 1] + C.bk[k + 1] * ps;
        st(delp, c0 + (long)k * G.lev, false, b64, bot - top);
        top = bot;
    }
}

template <class K, class... A>
void timed(const char *name, K kern, dim3 grd, dim3 blk, hipStream_t s, A... args)
{
    TimingRec r;
    bool tm = timing_wanted(name);
    if (tm) timing_begin(name, s, r);
    hipLaunchKernelGGL(kern, grd, blk, 0, s, args...);
    if (tm) timing_end(s, r);
}

}  // namespace

fv3_status run_remap(fv3_state *s, const fv3_grid *g, const double *ak, const double *bk, void *const *q,
                     int nq, hipStream_t st)
{
    const Geo &G = g->geo;
    const int n = g->n, nz = g->nz, b64 = g->bulk_bytes == 8;
    const double ptop = g->p.ptop;
    RCoef C{};
    for (int K = 0; K <= nz; K++) {
        C.ak[K] = ak[K];
        C.bk[K] = bk[K];
    }
    // workspace slots of one field each (FP64-sized, 256-byte aligned)
    const size_t slot = ((size_t)alloc_elems(g, nz) * 8 + 255) / 256 * 256;
    const int nslots = (int)std::min<size_t>(RSLOTS, s->workspace_bytes / slot);
    if (nslots < 2) return FV3_ESHAPE;
    char *ws = (char *)s->workspace;

    fv3_status hs = run_halo_cells(g, &s->delp, 1, nz, 0, st);   // face winds read the neighbour cells
    if (hs != FV3_OK) return hs;
    const dim3 blk(64, 4);
    // winds at faces
    {
        RBatch U{}, V{};
        U.src[0] = s->u;
        U.dst[0] = ws;
        U.nf = 1;
        V.src[0] = s->v;
        V.dst[0] = ws + slot;
        V.nf = 1;
        dim3 gu((unsigned)((n + 63) / 64), (unsigned)((n + 1 + 3) / 4), (unsigned)g->T);
        dim3 gv((unsigned)((n + 1 + 63) / 64), (unsigned)((n + 3) / 4), (unsigned)g->T);
        timed("k_remap_u", k_remap<RM_U, 1>, gu, blk, st, G, b64, ptop, C, U, (const void *)s->delp, g->flags);
        timed("k_remap_v", k_remap<RM_V, 1>, gv, blk, st, G, b64, ptop, C, V, (const void *)s->delp, g->flags);
        gu.z = (unsigned)(g->T * nz);
        gv.z = (unsigned)(g->T * nz);
        timed("k_remap_back", k_remap_back<RM_U>, gu, blk, st, G, b64, U);
        timed("k_remap_back", k_remap_back<RM_V>, gv, blk, st, G, b64, V);
    }
    // cell fields: pt, w, delz (as delz/delp), tracers, in batches of nslots
    std::vector<const void *> fs = {s->pt, s->w, s->delz};
    for (int m = 0; m < nq; m++) fs.push_back(q[m]);
    for (size_t b = 0; b < fs.size(); b += (size_t)nslots) {
        RBatch B{};
        B.nf = (int)std::min<size_t>((size_t)nslots, fs.size() - b);
        for (int f = 0; f < B.nf; f++) {
            B.src[f] = fs[b + f];
            B.dst[f] = ws + (size_t)f * slot;
            B.fp64[f] = fs[b + f] == (const void *)s->delz;
            B.ratio[f] = B.fp64[f];
        }
        const int groups = (B.nf + RNF - 1) / RNF;
        dim3 gc((unsigned)((n + 63) / 64), (unsigned)((n + 3) / 4), (unsigned)(g->T * groups));
        timed("k_remap_cells", k_remap<RM_CELL, RNF>, gc, blk, st, G, b64, ptop, C, B, (const void *)s->delp,
              g->flags);
        gc.z = (unsigned)(g->T * nz * B.nf);
        timed("k_remap_back", k_remap_back<RM_CELL>, gc, blk, st, G, b64, B);
    }
    dim3 gd((unsigned)((n + 63) / 64), (unsigned)((n + 3) / 4), (unsigned)g->T);
    timed("k_remap_delp", k_remap_delp, gd, blk, st, G, b64, ptop, C, s->delp);
    return hipGetLastError() == hipSuccess ? FV3_OK : FV3_EDEVICE;
}

}  // namespace fv3
