// Host-side grid construction: geometry, metric terms, tile connectivity and
// halo plans, then upload.  Runs once per grid (nothing here is hot).
//
// Cubed sphere (paper Sec. II): equiangular gnomonic projection of six cube
// faces; face t uses the frame (c, e1, e2) with e1 x e2 = c and places the
// lattice corner (I, J) at normalise(c + tan(a_I) e1 + tan(a_J) e2),
// a_I = (2I - n) pi / (4n).  The frame table below is a convention the
// initial-state generators use too.  Edges are matched between tiles by their
// midpoints; the lattice rotation between two tiles follows from the corner
// order, and gives the orientation transform of vector halos (Sec. V-C).
// Metric terms at halo points are those of the neighbour tile's own faces and
// cells (so halo stencils see exactly the neighbour's geometry); tile-edge
// faces carry cos = 0, sin = 1, which makes the normal wind there the stored
// wind (the tile-edge rule of Sec. V-B).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "fv3_internal.hpp"

namespace fv3 {
namespace {

struct V3 {
    double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) { return (1.0 / norm(a)) * a; }
inline double angle(V3 a, V3 b) { return std::atan2(norm(cross(a, b)), dot(a, b)); }
// unit vector in the tangent plane at p along chord d
inline V3 tangent(V3 p, V3 d) { return unit(d - dot(d, p) * p); }

const int kFrame[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},   {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {-1, 0, 0}, {0, -1, 0}}, {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},  {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

const int kSx[4] = {1, 0, 1, 0};
const int kSy[4] = {1, 1, 0, 0};

inline int fdiv2(int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); }

struct EdgeMap {
    int nb;
    int r[2][2];
    int ax2, ay2;   // doubled translation: q2 = R p2 + a2
};

class Geometry {
  public:
    Geometry(const fv3_grid_params &p) : P(p), n(p.n), cube(p.kind == FV3_GRID_CUBED_SPHERE) {}

    bool connect(std::string &err)
    {
        if (!cube) return true;
        // end points of edge e (W, E, S, N) in lattice units
        const int ends[4][2][2] = {{{0, 0}, {0, n}}, {{n, 0}, {n, n}}, {{0, 0}, {n, 0}}, {{0, n}, {n, n}}};
        for (int t = 0; t < 6; t++)
            for (int e = 0; e < 4; e++) {
                V3 mid = unit(corner(t, ends[e][0][0], ends[e][0][1]) + corner(t, ends[e][1][0], ends[e][1][1]));
                bool ok = false;
                for (int tb = 0; tb < 6 && !ok; tb++) {
                    if (tb == t) continue;
                    for (int eb = 0; eb < 4 && !ok; eb++) {
                        V3 mb = unit(corner(tb, ends[eb][0][0], ends[eb][0][1]) + corner(tb, ends[eb][1][0], ends[eb][1][1]));
                        if (angle(mid, mb) > 1e-9) continue;
                        // which end of eb coincides with our first end point
                        V3 a0 = corner(t, ends[e][0][0], ends[e][0][1]);
                        int o = angle(a0, corner(tb, ends[eb][0][0], ends[eb][0][1])) < 1e-9 ? 0 : 1;
                        const int *q0 = ends[eb][o], *q1 = ends[eb][1 - o];
                        int ta[2] = {(ends[e][1][0] - ends[e][0][0]) / n, (ends[e][1][1] - ends[e][0][1]) / n};
                        int tbv[2] = {(q1[0] - q0[0]) / n, (q1[1] - q0[1]) / n};
                        // proper rotation (det +1) taking ta to tbv: columns (ta -> tbv, perp(ta) -> perp(tbv))
                        int pa[2] = {-ta[1], ta[0]}, pb[2] = {-tbv[1], tbv[0]};
                        EdgeMap m;
                        m.nb = tb;
                        for (int r = 0; r < 2; r++)
                            for (int c = 0; c < 2; c++)
                                m.r[r][c] = tbv[r] * ta[c] + pb[r] * pa[c];
                        m.ax2 = 2 * q0[0] - (m.r[0][0] * 2 * ends[e][0][0] + m.r[0][1] * 2 * ends[e][0][1]);
                        m.ay2 = 2 * q0[1] - (m.r[1][0] * 2 * ends[e][0][0] + m.r[1][1] * 2 * ends[e][0][1]);
                        em[t][e] = m;
                        ok = true;
                    }
                }
                if (!ok) {
                    err = "cube connectivity: tile " + std::to_string(t) + " edge " + std::to_string(e);
                    return false;
                }
            }
        return true;
    }

    // Unit-sphere position of lattice corner (I, J) of tile t (interior range).
    V3 corner(int t, int I, int J) const
    {
        double ta = I == 0 ? -1.0 : (I == n ? 1.0 : std::tan((2 * I - n) * M_PI / (4.0 * n)));
        double tb = J == 0 ? -1.0 : (J == n ? 1.0 : std::tan((2 * J - n) * M_PI / (4.0 * n)));
        V3 c{(double)kFrame[t][0][0], (double)kFrame[t][0][1], (double)kFrame[t][0][2]};
        V3 a{(double)kFrame[t][1][0], (double)kFrame[t][1][1], (double)kFrame[t][1][2]};
        V3 b{(double)kFrame[t][2][0], (double)kFrame[t][2][1], (double)kFrame[t][2][2]};
        return unit(c + ta * a + tb * b);
    }

    // region of doubled point: 0 interior, 1 edge halo, 2 corner block
    int region(int x2, int y2) const
    {
        bool ix = x2 >= 0 && x2 <= 2 * n, iy = y2 >= 0 && y2 <= 2 * n;
        return (ix && iy) ? 0 : ((ix || iy) ? 1 : 2);
    }

    // Map an edge-halo point (or, periodic, any halo point) to its owner.
    void owner(int t, int x2, int y2, int &tb, int &qx2, int &qy2, int r[2][2]) const
    {
        int n2 = 2 * n;
        if (!cube) {
            tb = t;
            qx2 = x2 < 0 ? x2 + n2 : (x2 > n2 ? x2 - n2 : x2);
            qy2 = y2 < 0 ? y2 + n2 : (y2 > n2 ? y2 - n2 : y2);
            r[0][0] = r[1][1] = 1;
            r[0][1] = r[1][0] = 0;
            return;
        }
        int e = x2 < 0 ? 0 : (x2 > n2 ? 1 : (y2 < 0 ? 2 : 3));
        const EdgeMap &m = em[t][e];
        tb = m.nb;
        std::memcpy(r, m.r, sizeof(m.r));
        qx2 = m.r[0][0] * x2 + m.r[0][1] * y2 + m.ax2;
        qy2 = m.r[1][0] * x2 + m.r[1][1] * y2 + m.ay2;
    }

    // The affine map of edge e of tile t applied to a point (doubled lattice
    // coordinates) on that edge: the same point in the neighbour tile.
    void edge_map(int t, int e, int x2, int y2, int &tb, int &qx2, int &qy2, int r[2][2]) const
    {
        const EdgeMap &m = em[t][e];
        tb = m.nb;
        std::memcpy(r, m.r, sizeof(m.r));
        qx2 = m.r[0][0] * x2 + m.r[0][1] * y2 + m.ax2;
        qy2 = m.r[1][0] * x2 + m.r[1][1] * y2 + m.ay2;
    }

    // Position of lattice corner (I, J) of tile t, halo corners via the owner.
    V3 corner_ext(int t, int I, int J) const
    {
        if (region(2 * I, 2 * J) == 0) return corner(t, I, J);
        int tb, qx, qy, r[2][2];
        owner(t, 2 * I, 2 * J, tb, qx, qy, r);
        return corner(tb, qx / 2, qy / 2);
    }
    V3 centre_ext(int t, int i, int j) const
    {
        return unit(corner_ext(t, i, j) + corner_ext(t, i + 1, j) + corner_ext(t, i + 1, j + 1) +
                    corner_ext(t, i, j + 1));
    }

    // Metric term m of the point of its staggering at (i, j) of tile t.
    double metric(int m, int t, int i, int j) const
    {
        static const int stag[M_COUNT] = {SY, SX, SX, SY, SC, SC, SC, SB, SC, SB, SX, SX, SY, SY, SC, SC};
        int st = stag[m];
        int x2 = 2 * i + kSx[st], y2 = 2 * j + kSy[st];
        if (!cube) return periodic_metric(m);
        int reg = region(x2, y2);
        if (reg == 2) return std::numeric_limits<double>::quiet_NaN();
        if (reg == 1) {
            int tb, qx, qy, r[2][2];
            owner(t, x2, y2, tb, qx, qy, r);
            bool swap = r[0][0] == 0;
            int sx = r[0][0] + r[1][0], sy = r[0][1] + r[1][1];   // signs of our x and y images
            static const int partner[M_COUNT] = {M_DY, M_DX, M_DYC, M_DXC, M_DYA, M_DXA, M_AREA, M_AREA_C, M_FC,
                                                 M_FB, M_SIN_V, M_COS_V, M_SIN_U, M_COS_U, M_SIN_A, M_COS_A};
            int mm = swap ? partner[m] : m;
            double v = interior_metric(mm, tb, fdiv2(qx), fdiv2(qy));
            if (m == M_COS_U || m == M_COS_V || m == M_COS_A) v *= (double)(sx * sy);
            return v;
        }
        return interior_metric(m, t, i, j);
    }

  private:
    double periodic_metric(int m) const
    {
        double d = P.dx;
        switch (m) {
        case M_AREA: case M_AREA_C: return d * d;
        case M_FC: case M_FB: return P.f0;
        case M_SIN_U: case M_SIN_V: case M_SIN_A: return 1.0;
        case M_COS_U: case M_COS_V: case M_COS_A: return 0.0;
        default: return d;
        }
    }

    // excess of the spherical quadrilateral a b c d: sum of (angle - pi/2)
    static double quad_excess(V3 a, V3 b, V3 c, V3 d)
    {
        V3 v[4] = {a, b, c, d};
        double s = 0;
        for (int k = 0; k < 4; k++) {
            V3 p = v[k], t1 = tangent(p, v[(k + 3) % 4] - p), t2 = tangent(p, v[(k + 1) % 4] - p);
            s -= std::atan2(dot(t1, t2), norm(cross(t1, t2)));
        }
        return s;
    }
    static double tri_excess(V3 a, V3 b, V3 c)
    {
        return 2.0 * std::atan2(std::fabs(dot(a, cross(b, c))), 1.0 + dot(a, b) + dot(b, c) + dot(c, a));
    }

    double interior_metric(int m, int t, int i, int j) const
    {
        double a = P.radius;
        switch (m) {
        case M_DX: return a * angle(corner(t, i, j), corner(t, i + 1, j));
        case M_DY: return a * angle(corner(t, i, j), corner(t, i, j + 1));
        case M_DXC: return a * angle(centre_ext(t, i - 1, j), centre_ext(t, i, j));
        case M_DYC: return a * angle(centre_ext(t, i, j - 1), centre_ext(t, i, j));
        case M_DXA: return a * angle(xmid(t, i, j), xmid(t, i + 1, j));
        case M_DYA: return a * angle(ymid(t, i, j), ymid(t, i, j + 1));
        case M_AREA:
            return a * a * quad_excess(corner(t, i, j), corner(t, i + 1, j), corner(t, i + 1, j + 1), corner(t, i, j + 1));
        case M_AREA_C: {
            bool vx = (i == 0 || i == n), vy = (j == 0 || j == n);
            if (vx && vy) {
                // cube vertex: three cells meet; drop the one in the missing corner block
                V3 c[4];
                int ci[4][2] = {{i - 1, j - 1}, {i, j - 1}, {i, j}, {i - 1, j}};
                int k = 0;
                for (int q = 0; q < 4; q++) {
                    int x2 = 2 * ci[q][0] + 1, y2 = 2 * ci[q][1] + 1;
                    if (region(x2, y2) == 2) continue;
                    c[k++] = centre_ext(t, ci[q][0], ci[q][1]);
                }
                return a * a * tri_excess(c[0], c[1], c[2]);
            }
            return a * a * quad_excess(centre_ext(t, i - 1, j - 1), centre_ext(t, i, j - 1), centre_ext(t, i, j),
                                       centre_ext(t, i - 1, j));
        }
        case M_FC: return 2.0 * P.omega * centre_ext(t, i, j).z;
        case M_FB: return 2.0 * P.omega * corner(t, i, j).z;
        case M_SIN_U: case M_COS_U: {
            if (i == 0 || i == n) return m == M_SIN_U ? 1.0 : 0.0;
            V3 mid = xmid(t, i, j);
            V3 ey = tangent(mid, corner(t, i, j + 1) - corner(t, i, j));
            V3 ex = tangent(mid, centre_ext(t, i, j) - centre_ext(t, i - 1, j));
            double c = dot(ex, ey);
            return m == M_COS_U ? c : std::sqrt(1.0 - c * c);
        }
        case M_SIN_V: case M_COS_V: {
            if (j == 0 || j == n) return m == M_SIN_V ? 1.0 : 0.0;
            V3 mid = ymid(t, i, j);
            V3 ex = tangent(mid, corner(t, i + 1, j) - corner(t, i, j));
            V3 ey = tangent(mid, centre_ext(t, i, j) - centre_ext(t, i, j - 1));
            double c = dot(ex, ey);
            return m == M_COS_V ? c : std::sqrt(1.0 - c * c);
        }
        case M_SIN_A: case M_COS_A: {
            V3 p = centre_ext(t, i, j);
            V3 ex = tangent(p, xmid(t, i + 1, j) - xmid(t, i, j));
            V3 ey = tangent(p, ymid(t, i, j + 1) - ymid(t, i, j));
            double c = dot(ex, ey);
            return m == M_COS_A ? c : std::sqrt(1.0 - c * c);
        }
        }
        return 0.0;
    }
    V3 xmid(int t, int i, int j) const { return unit(corner(t, i, j) + corner(t, i, j + 1)); }
    V3 ymid(int t, int i, int j) const { return unit(corner(t, i, j) + corner(t, i + 1, j)); }

  public:
    const fv3_grid_params &P;
    int n;
    bool cube;
    EdgeMap em[6][4];
};

template <class T>
fv3_status upload(T **dst, const std::vector<T> &h, std::string &err)
{
    if (hipMalloc((void **)dst, h.size() * sizeof(T)) != hipSuccess) {
        err = "hipMalloc failed";
        return FV3_ENOMEM;
    }
    if (hipMemcpy(*dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMemcpy failed";
        return FV3_EDEVICE;
    }
    return FV3_OK;
}

// Halo plan for one staggering (scalar) or a pair of staggerings (vector).
void make_plan(const Geometry &G, const fv3_grid *g, int stx, int sty, bool pair,
               std::vector<HaloEnt> &out)
{
    int n = G.n;
    for (int comp = 0; comp < (pair ? 2 : 1); comp++) {
        int st = comp == 0 ? stx : sty;
        int ihi = (st == SX || st == SB) ? n + HALO : n + HALO - 1;
        int jhi = (st == SY || st == SB) ? n + HALO : n + HALO - 1;
        for (int t = 0; t < g->T; t++)
            for (int j = -HALO; j <= jhi; j++)
                for (int i = -HALO; i <= ihi; i++) {
                    int x2 = 2 * i + kSx[st], y2 = 2 * j + kSy[st];
                    int reg = G.region(x2, y2);
                    if (reg == 0 || (reg == 2 && G.cube)) continue;
                    int tb, qx, qy, r[2][2];
                    G.owner(t, x2, y2, tb, qx, qy, r);
                    int sel = comp ? 4 : 0;
                    if (pair) {
                        // our direction (comp) maps to the neighbour's column of R
                        int vx = comp == 0 ? r[0][0] : r[0][1];
                        int vy = comp == 0 ? r[1][0] : r[1][1];
                        int src_comp = vx != 0 ? 0 : 1;
                        int sgn = vx != 0 ? vx : vy;
                        sel |= src_comp | (sgn < 0 ? 2 : 0);
                    }
                    HaloEnt h;
                    h.dt = t;
                    h.di = (int)((long)j * g->pitch + i);
                    h.st = tb;
                    h.si = (int)((long)fdiv2(qy) * g->pitch + fdiv2(qx));
                    h.sel = sel;
                    out.push_back(h);
                }
    }
}

// Edge cells of the cube for the edge-flux fix-up: every cell with a face on
// a tile edge, each such face with its partner copy on the neighbour tile.
bool make_edge_cells(const Geometry &G, const fv3_grid *g, std::vector<EdgeCell> &out)
{
    if (!G.cube) return true;
    const int n = G.n;
    for (int t = 0; t < g->T; t++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                if (i > 0 && i < n - 1 && j > 0 && j < n - 1) continue;
                EdgeCell c{};
                c.t = t;
                c.cell = (int)((long)j * g->pitch + i);
                // (edge, face stagger x = 0 / y = 1, face i, j, inflow sign)
                int faces[4][5], m = 0;
                if (i == 0) { int f[5] = {0, 0, 0, j, 1}; std::memcpy(faces[m++], f, sizeof(f)); }
                if (i == n - 1) { int f[5] = {1, 0, n, j, -1}; std::memcpy(faces[m++], f, sizeof(f)); }
                if (j == 0) { int f[5] = {2, 1, i, 0, 1}; std::memcpy(faces[m++], f, sizeof(f)); }
                if (j == n - 1) { int f[5] = {3, 1, i, n, -1}; std::memcpy(faces[m++], f, sizeof(f)); }
                c.nf = m;
                for (int q = 0; q < m; q++) {
                    const int e = faces[q][0], ax = faces[q][1], fi = faces[q][2], fj = faces[q][3];
                    const int x2 = 2 * fi + (ax == 0 ? 0 : 1), y2 = 2 * fj + (ax == 0 ? 1 : 0);
                    int tb, qx2, qy2, r[2][2];
                    G.edge_map(t, e, x2, y2, tb, qx2, qy2, r);
                    // our normal direction (x for x-faces, y for y-faces) in the neighbour's frame
                    const int vx = ax == 0 ? r[0][0] : r[0][1], vy = ax == 0 ? r[1][0] : r[1][1];
                    c.arr[q] = ax;
                    c.off[q] = (int)((long)fj * g->pitch + fi);
                    c.sin[q] = faces[q][4];
                    c.pt[q] = tb;
                    c.parr[q] = vx != 0 ? 0 : 1;
                    c.spar[q] = vx != 0 ? vx : vy;
                    // the partner is a face on one of the neighbour's edges
                    const int pi = fdiv2(qx2), pj = fdiv2(qy2);
                    const bool xf = (qx2 & 1) == 0 && (qy2 & 1) == 1, yf = (qx2 & 1) == 1 && (qy2 & 1) == 0;
                    if (tb < 0 || tb >= g->T || pi < 0 || pi > n || pj < 0 || pj > n || !(xf || yf) ||
                        (xf && pi != 0 && pi != n) || (yf && pj != 0 && pj != n) || xf != (c.parr[q] == 0))
                        return false;
                    c.poff[q] = (int)((long)pj * g->pitch + pi);
                }
                out.push_back(c);
            }
    return true;
}

}  // namespace

static void set_layout(const fv3_grid_params *p, fv3_grid *g)
{
    g->p = *p;
    g->n = p->n;
    g->nz = p->nz;
    g->T = p->kind == FV3_GRID_CUBED_SPHERE ? 6 : 1;
    int align = p->precision == FV3_MIXED ? 32 : 16;   // elements per 128 bytes of the bulk type
    g->rows = p->n + 2 * HALO + 1;
    g->pitch = (g->rows + align - 1) / align * align;
    g->lev = g->rows * g->pitch;
    g->pre = align - HALO;
    g->off0 = g->pre + HALO + (long)HALO * g->pitch;
    g->bulk_bytes = p->precision == FV3_MIXED ? 4 : 8;
    g->geo = Geo{g->n, g->nz, g->T, p->kind == FV3_GRID_CUBED_SPHERE ? 1 : 0, g->pitch, g->lev, g->off0};
}

static const int kMetricStag[M_COUNT] = {SY, SX, SX, SY, SC, SC, SC, SB, SC, SB, SX, SX, SY, SY, SC, SC};

// metric m on every storage point of its staggering, in the field layout (L = 1)
static void fill_metric(const Geometry &G, const fv3_grid *g, int m, std::vector<double> &h)
{
    h.assign(alloc_elems(g, 1), 0.0);
    int st = kMetricStag[m];
    int ihi = (st == SX || st == SB) ? g->n + HALO : g->n + HALO - 1;
    int jhi = (st == SY || st == SB) ? g->n + HALO : g->n + HALO - 1;
    for (int t = 0; t < g->T; t++)
        for (int j = -HALO; j <= jhi; j++)
            for (int i = -HALO; i <= ihi; i++) {
                double v = G.metric(m, t, i, j);
                if (std::isnan(v)) v = 0.0;   // cube corner blocks: never read directly
                h[g->off0 + (long)t * g->lev + (long)j * g->pitch + i] = v;
            }
}

fv3_status host_metric(const fv3_grid_params *p, int m, double *out, long cap, std::string &err)
{
    fv3_grid g;
    set_layout(p, &g);
    long N = g.rows;
    if (cap < (long)g.T * N * N) {
        err = "output too small";
        return FV3_ESHAPE;
    }
    Geometry G(g.p);
    if (!G.connect(err)) return FV3_EINTERNAL;
    std::vector<double> h;
    fill_metric(G, &g, m, h);
    for (int t = 0; t < g.T; t++)
        for (long jj = 0; jj < N; jj++)
            for (long ii = 0; ii < N; ii++)
                out[((long)t * N + jj) * N + ii] = h[g.pre + (long)t * g.lev + jj * g.pitch + ii];
    return FV3_OK;
}

fv3_status build_grid(const fv3_grid_params *p, fv3_grid *g, std::string &err)
{
    set_layout(p, g);
    Geometry G(g->p);
    if (!G.connect(err)) return FV3_EINTERNAL;
    for (int m = 0; m < M_COUNT; m++) fill_metric(G, g, m, g->hmet[m]);
    {
        // derived reciprocals: base term and power
        static const int base[M_ALL - M_COUNT] = {M_DX, M_DY, M_DXC, M_DYC, M_AREA, M_AREA_C,
                                                  M_SIN_U, M_SIN_V, M_SIN_A};
        static const int pw[M_ALL - M_COUNT] = {1, 1, 1, 1, 1, 1, 1, 1, 2};
        for (int m = M_COUNT; m < M_ALL; m++) {
            const std::vector<double> &b = g->hmet[base[m - M_COUNT]];
            std::vector<double> &h = g->hmet[m];
            h.assign(b.size(), 0.0);
            for (size_t e = 0; e < b.size(); e++) {
                double x = pw[m - M_COUNT] == 2 ? b[e] * b[e] : b[e];
                h[e] = x != 0.0 ? 1.0 / x : 0.0;
            }
        }
    }
    for (int m = 0; m < M_ALL; m++) {
        std::vector<double> &h = g->hmet[m];
        fv3_status s = upload(&g->met[m], h, err);
        if (s != FV3_OK) return s;
        if (p->precision == FV3_MIXED) {
            std::vector<float> f(h.begin(), h.end());
            s = upload(&g->metf[m], f, err);
            if (s != FV3_OK) return s;
        }
    }
    {
        const std::vector<double> &ac = g->hmet[M_AREA_C];
        double m = 1e300;
        for (int t = 0; t < g->T; t++)
            for (int j = 0; j <= g->n; j++)
                for (int i = 0; i <= g->n; i++)
                    m = std::min(m, ac[g->off0 + (long)t * g->lev + (long)j * g->pitch + i]);
        g->da_min = m;
    }
    std::vector<HaloEnt> pc, pd, pcv, pa, pb;
    make_plan(G, g, SC, SC, false, pc);
    make_plan(G, g, SB, SB, false, pb);   // corner scalar
    make_plan(G, g, SC, SC, true, pa);    // cell-centred vector
    make_plan(G, g, SY, SX, true, pd);    // D grid: u (x comp) on y-faces, v on x-faces
    make_plan(G, g, SX, SY, true, pcv);   // C grid: uc on x-faces, vc on y-faces
    fv3_status s;
    if ((s = upload(&g->planC.d, pc, err)) != FV3_OK) return s;
    g->planC.count = (int)pc.size();
    if ((s = upload(&g->planD.d, pd, err)) != FV3_OK) return s;
    g->planD.count = (int)pd.size();
    if ((s = upload(&g->planCv.d, pcv, err)) != FV3_OK) return s;
    g->planCv.count = (int)pcv.size();
    if ((s = upload(&g->planA.d, pa, err)) != FV3_OK) return s;
    g->planA.count = (int)pa.size();
    if ((s = upload(&g->planB.d, pb, err)) != FV3_OK) return s;
    g->planB.count = (int)pb.size();
    std::vector<EdgeCell> ec;
    if (!make_edge_cells(G, g, ec)) {
        err = "edge-cell plan: a tile-edge face has no partner face on the neighbour's edge";
        return FV3_EINTERNAL;
    }
    if (!ec.empty()) {
        if ((s = upload(&g->edge_cells, ec, err)) != FV3_OK) return s;
        g->edge_count = (int)ec.size();
    }
    if (hipMalloc((void **)&g->flags, 4 * sizeof(int)) != hipSuccess) return FV3_ENOMEM;
    if (hipMemset(g->flags, 0, 4 * sizeof(int)) != hipSuccess) return FV3_EDEVICE;
    return FV3_OK;
}

}  // namespace fv3
