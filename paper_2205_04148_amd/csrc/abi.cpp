// C ABI entry points: argument validation, grid lifetime, error reporting.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "fv3_internal.hpp"

namespace {
thread_local std::string g_last_error;

fv3_status fail(fv3_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

bool device_ok(const fv3_grid *g)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return false;
    return cur == g->p.device;
}

fv3_status check_state(const fv3_state *s, const fv3_grid *g)
{
    if (!s || !g) return fail(FV3_EINVAL, "NULL state or grid");
    const void *req[] = {s->u, s->v, s->w, s->delp, s->pt, s->delz, s->uc, s->vc, s->mfx, s->mfy,
                         s->cx, s->cy, s->dp0, s->pfull, s->phi, s->workspace};
    for (const void *p : req)
        if (!p) return fail(FV3_EINVAL, "NULL field in fv3_state");
    if (s->workspace_bytes < g->ws_bytes)
        return fail(FV3_EINVAL, "workspace too small: need " + std::to_string(g->ws_bytes) + " bytes");
    if (!device_ok(g)) return fail(FV3_EDEVICE, "current HIP device differs from the grid's device");
    return FV3_OK;
}
fv3_status check_remap_coeffs(const fv3_grid *g, const double *ak, const double *bk)
{
    const int nz = g->nz;
    if (nz > FV3_REMAP_MAX_LEVELS) return fail(FV3_ESHAPE, "nz exceeds FV3_REMAP_MAX_LEVELS");
    for (int K = 0; K <= nz; K++)
        if (!std::isfinite(ak[K]) || !std::isfinite(bk[K])) return fail(FV3_EINVAL, "non-finite ak or bk");
    if (ak[0] != g->p.ptop || bk[0] != 0.0 || ak[nz] != 0.0 || bk[nz] != 1.0)
        return fail(FV3_EINVAL, "need ak[0] = ptop, bk[0] = 0, ak[nz] = 0, bk[nz] = 1");
    return FV3_OK;
}
}  // namespace

namespace fv3 {
fv3_status set_error(fv3_status s, const std::string &msg) { return fail(s, msg); }
bool device_current(const fv3_grid *g) { return device_ok(g); }
}  // namespace fv3

extern "C" {

const char *fv3_last_error(void) { return g_last_error.c_str(); }

const char *fv3_status_string(fv3_status s)
{
    switch (s) {
    case FV3_OK: return "ok";
    case FV3_EINVAL: return "invalid argument";
    case FV3_ESHAPE: return "inconsistent sizes";
    case FV3_EDTYPE: return "precision mismatch";
    case FV3_EDEVICE: return "HIP device error";
    case FV3_ENOMEM: return "out of device memory";
    case FV3_ECFL: return "Courant number above 1";
    case FV3_ENONFINITE: return "non-finite prognostic";
    case FV3_EUNSUPPORTED: return "unsupported option";
    case FV3_EREMAP: return "reference interfaces not increasing";
    case FV3_EINTERNAL: return "internal error";
    }
    return "unknown status";
}

fv3_status fv3_init_grid(const fv3_grid_params *p, fv3_grid **out)
{
    if (!p || !out) return fail(FV3_EINVAL, "NULL params or output");
    *out = nullptr;
    if (p->kind != FV3_GRID_DOUBLY_PERIODIC && p->kind != FV3_GRID_CUBED_SPHERE)
        return fail(FV3_EINVAL, "unknown grid kind");
    if (p->n < 8 || p->n > 4096 || p->nz < 1 || p->nz > 512)
        return fail(FV3_ESHAPE, "n must be in [8, 4096] and nz in [1, 512]");
    if (p->precision != FV3_FP64 && p->precision != FV3_MIXED) return fail(FV3_EDTYPE, "unknown precision");
    if (p->hord != 8 && p->hord != 6 && p->hord != 5)
        return fail(FV3_EUNSUPPORTED, "PPM order hord must be 8 (monotone), 6 (unlimited) or 5 (2dx-filtered)");
    if (p->hord_tr != 0 && p->hord_tr != 5 && p->hord_tr != 6 && p->hord_tr != 7 && p->hord_tr != 8)
        return fail(FV3_EUNSUPPORTED, "tracer PPM order hord_tr must be 0 (= hord), 5, 6, 7 or 8");
    if (p->nord < 0 || p->nord > 2) return fail(FV3_EUNSUPPORTED, "nord must be 0, 1 (del-4) or 2 (del-6)");
    if (!std::isfinite(p->d4_bg) || p->d4_bg < 0.0 || p->d4_bg > 0.25)
        return fail(FV3_EINVAL, "d4_bg must be in [0, 0.25]");
    if (p->edge_fix != 0 && p->edge_fix != 1) return fail(FV3_EINVAL, "edge_fix must be 0 or 1");
    if (p->edge_ppm != 0 && p->edge_ppm != 1) return fail(FV3_EINVAL, "edge_ppm must be 0 or 1");
    if (p->edge_interp != 0 && p->edge_interp != 1) return fail(FV3_EINVAL, "edge_interp must be 0 or 1");
    if (!std::isfinite(p->vtdm) || p->vtdm < 0.0 || p->vtdm > 0.25)
        return fail(FV3_EINVAL, "vtdm must be in [0, 0.25]");
    if (p->pp_order != 0 && p->pp_order != 2 && p->pp_order != 4)
        return fail(FV3_EUNSUPPORTED, "pp_order must be 2 (mass-linear; 0 means the same) or 4 (cubic)");
    if (!(p->d2_bg >= 0.0 && p->d2_bg <= 0.25))
        return fail(FV3_EINVAL, "d2_bg must be in [0, 0.25] (explicit del-2 damping)");
    if (!(p->dddmp >= 0.0 && p->dddmp <= 1.0))
        return fail(FV3_EINVAL, "dddmp (Smagorinsky divergence damping) must be in [0, 1]");
    if (!(p->beta >= 0.5 && p->beta <= 1.0))
        return fail(FV3_EINVAL, "beta (off-centring of the vertical solve) must be in [0.5, 1]");
    if (!(p->ptop > 0.0) || !std::isfinite(p->ptop)) return fail(FV3_EINVAL, "ptop must be positive");
    if (p->kind == FV3_GRID_DOUBLY_PERIODIC && !(p->dx > 0.0)) return fail(FV3_EINVAL, "dx must be positive");
    if (p->kind == FV3_GRID_CUBED_SPHERE && !(p->radius > 0.0)) return fail(FV3_EINVAL, "radius must be positive");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || p->device < 0 || p->device >= ndev)
        return fail(FV3_EDEVICE, "no such HIP device");
    if (hipSetDevice(p->device) != hipSuccess) return fail(FV3_EDEVICE, "hipSetDevice failed");
    fv3_grid *g = new (std::nothrow) fv3_grid();
    if (!g) return fail(FV3_ENOMEM, "host allocation failed");
    std::string err;
    fv3_status s = fv3::build_grid(p, g, err);
    if (s != FV3_OK) {
        fv3_free_grid(g);
        return fail(s, "grid construction: " + err);
    }
    // the allocation-free entry point's scratch address on this device
    // (hipSetDevice above made it current)
    if (fv3::noalloc_setup(p->device) != FV3_OK) {
        fv3_free_grid(g);
        return fail(FV3_EDEVICE, "hipGetSymbolAddress of the fixed scratch array failed");
    }
    g->ws_bytes = fv3::workspace_bytes(g);
    g->red_elems = fv3::reduction_elems(g);
    if (hipMalloc((void **)&g->red, g->red_elems * sizeof(double)) != hipSuccess) {
        fv3_free_grid(g);
        return fail(FV3_ENOMEM, "reduction scratch allocation failed");
    }
    *out = g;
    return FV3_OK;
}

fv3_status fv3_free_grid(fv3_grid *g)
{
    if (!g) return FV3_OK;
    (void)hipDeviceSynchronize();
    for (int m = 0; m < fv3::M_ALL; m++) {
        if (g->met[m]) (void)hipFree(g->met[m]);
        if (g->metf[m]) (void)hipFree(g->metf[m]);
    }
    if (g->planC.d) (void)hipFree(g->planC.d);
    if (g->planD.d) (void)hipFree(g->planD.d);
    if (g->planCv.d) (void)hipFree(g->planCv.d);
    if (g->planA.d) (void)hipFree(g->planA.d);
    if (g->planB.d) (void)hipFree(g->planB.d);
    if (g->edge_cells) (void)hipFree(g->edge_cells);
    if (g->flags) (void)hipFree(g->flags);
    if (g->red) (void)hipFree(g->red);
    delete g;
    return FV3_OK;
}

fv3_status fv3_grid_layout(const fv3_grid *g, fv3_layout *out)
{
    if (!g || !out) return fail(FV3_EINVAL, "NULL grid or output");
    out->tiles = g->T;
    out->n = g->n;
    out->nz = g->nz;
    out->halo = fv3::HALO;
    out->pitch = g->pitch;
    out->rows = g->rows;
    out->level_elems = g->lev;
    out->offset0 = g->off0;
    out->bulk_elem_bytes = g->bulk_bytes;
    return FV3_OK;
}

size_t fv3_workspace_bytes(const fv3_grid *g) { return g ? g->ws_bytes : 0; }

fv3_status fv3_grid_metric(const fv3_grid *g, int which, double *host_out)
{
    if (!g || !host_out) return fail(FV3_EINVAL, "NULL grid or output");
    if (which < 0 || which >= fv3::M_COUNT) return fail(FV3_EINVAL, "metric index out of range");
    std::memcpy(host_out, g->hmet[which].data(), g->hmet[which].size() * sizeof(double));
    return FV3_OK;
}

fv3_status fv3_host_grid_metric(const fv3_grid_params *p, int which, double *host_out, long max_elems)
{
    if (!p || !host_out) return fail(FV3_EINVAL, "NULL params or output");
    if (which < 0 || which >= fv3::M_COUNT) return fail(FV3_EINVAL, "metric index out of range");
    if (p->kind != FV3_GRID_DOUBLY_PERIODIC && p->kind != FV3_GRID_CUBED_SPHERE)
        return fail(FV3_EINVAL, "unknown grid kind");
    if (p->n < 8 || p->n > 4096 || p->nz < 1) return fail(FV3_ESHAPE, "bad sizes");
    std::string err;
    fv3_status s = fv3::host_metric(p, which, host_out, max_elems, err);
    if (s != FV3_OK) return fail(s, err);
    return FV3_OK;
}

static fv3_status substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split, int stop,
                           void *stream)
{
    fv3_status st = check_state(s, g);
    if (st != FV3_OK) return st;
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(FV3_EINVAL, "dt must be finite and positive");
    if (n_split < 1) return fail(FV3_EINVAL, "n_split must be >= 1");
    st = fv3::run_substeps(s, g, dt, n_split, stop, (hipStream_t)stream);
    if (st != FV3_OK) return fail(st, "substep launch failed");
    return FV3_OK;
}

fv3_status fv3_acoustic_substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split, void *stream)
{
    return substeps(s, g, dt, n_split, 0, stream);
}

fv3_status fv3_acoustic_substeps_debug(fv3_state *s, const fv3_grid *g, double dt, int n_split,
                                       int stop_stage, void *stream)
{
    if (stop_stage < 0 || stop_stage > 10) return fail(FV3_EINVAL, "stop_stage out of range");
    return substeps(s, g, dt, n_split, stop_stage, stream);
}

fv3_status fv3_tracer_transport(void *const *q, int nq, fv3_state *s, const fv3_grid *g, int nsplt,
                                void *stream)
{
    if (!q || nq < 1 || nq > 64) return fail(FV3_EINVAL, "need 1..64 tracers");
    for (int m = 0; m < nq; m++)
        if (!q[m]) return fail(FV3_EINVAL, "NULL tracer pointer");
    fv3_status st = check_state(s, g);
    if (st != FV3_OK) return st;
    if (nsplt > FV3_MAX_TRACER_SUBCYCLES)
        return fail(FV3_EINVAL, "nsplt above FV3_MAX_TRACER_SUBCYCLES (" +
                                    std::to_string(FV3_MAX_TRACER_SUBCYCLES) + ")");
    st = fv3::run_tracer(q, nq, s, g, nsplt, (hipStream_t)stream);
    if (st == FV3_ENONFINITE || st == FV3_ECFL) return st;   // message set where it was found
    if (st != FV3_OK) return fail(st, "tracer transport failed");
    return FV3_OK;
}

fv3_status fv3_remap(fv3_state *s, const fv3_grid *g, const double *ak, const double *bk, void *const *q,
                     int nq, void *stream)
{
    if (!ak || !bk) return fail(FV3_EINVAL, "NULL ak or bk");
    if (nq < 0 || nq > 64 || (nq > 0 && !q)) return fail(FV3_EINVAL, "need 0..64 tracers");
    for (int m = 0; m < nq; m++)
        if (!q[m]) return fail(FV3_EINVAL, "NULL tracer pointer");
    fv3_status st = check_state(s, g);
    if (st != FV3_OK) return st;
    st = check_remap_coeffs(g, ak, bk);
    if (st != FV3_OK) return st;
    st = fv3::run_remap(s, g, ak, bk, q, nq, (hipStream_t)stream);
    if (st != FV3_OK) return fail(st, "remap failed");
    return FV3_OK;
}

fv3_status fv3_dynamics(fv3_state *s, const fv3_grid *g, void *const *q, int nq, const double *ak,
                        const double *bk, double dt, int k_split, int n_split, int nsplt, void *stream)
{
    if (!ak || !bk) return fail(FV3_EINVAL, "NULL ak or bk");
    if (nq < 0 || nq > 64 || (nq > 0 && !q)) return fail(FV3_EINVAL, "need 0..64 tracers");
    for (int m = 0; m < nq; m++)
        if (!q[m]) return fail(FV3_EINVAL, "NULL tracer pointer");
    fv3_status st = check_state(s, g);
    if (st != FV3_OK) return st;
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(FV3_EINVAL, "dt must be finite and positive");
    if (k_split < 1 || n_split < 1) return fail(FV3_EINVAL, "k_split and n_split must be >= 1");
    if (nsplt > FV3_MAX_TRACER_SUBCYCLES)
        return fail(FV3_EINVAL, "nsplt above FV3_MAX_TRACER_SUBCYCLES");
    st = check_remap_coeffs(g, ak, bk);
    if (st != FV3_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    const double dtk = dt / k_split;
    for (int it = 0; it < k_split; it++) {
        st = fv3::run_substeps(s, g, dtk, n_split, 0, hs);
        if (st != FV3_OK) return fail(st, "substep launch failed");
        if (nq > 0) {
            st = fv3::run_tracer(q, nq, s, g, nsplt, hs);
            if (st == FV3_ENONFINITE || st == FV3_ECFL) return st;
            if (st != FV3_OK) return fail(st, "tracer transport failed");
        }
        st = fv3::run_remap(s, g, ak, bk, q, nq, hs);
        if (st != FV3_OK) return fail(st, "remap failed");
    }
    return FV3_OK;
}

fv3_status fv3_mass_sums(const fv3_grid *g, const void *delp, const void *pt, void *const *q, int nq,
                         double *host_out, void *stream)
{
    if (!g || !delp || !pt || !host_out || nq < 0 || (nq > 0 && !q))
        return fail(FV3_EINVAL, "NULL argument");
    for (int m = 0; m < nq; m++)
        if (!q[m]) return fail(FV3_EINVAL, "NULL tracer pointer");
    if (!device_ok(g)) return fail(FV3_EDEVICE, "current HIP device differs from the grid's device");
    static std::mutex mu;   // the grid's reduction scratch is shared
    std::lock_guard<std::mutex> lock(mu);
    fv3_status st = fv3::run_mass_sums(g, delp, pt, q, nq, host_out, (hipStream_t)stream);
    if (st != FV3_OK) return fail(st, "mass sums failed");
    return FV3_OK;
}

fv3_status fv3_mass_sums_noalloc(const fv3_grid *g, const void *delp, const void *pt, void *const *q, int nq,
                                 double *dev_out, void *stream)
{
    if (!g || !delp || !pt || !dev_out || nq < 0 || (nq > 0 && !q))
        return fail(FV3_EINVAL, "NULL argument");
    if (nq > 64) return fail(FV3_EINVAL, "need 0..64 tracers");
    for (int m = 0; m < nq; m++)
        if (!q[m]) return fail(FV3_EINVAL, "NULL tracer pointer");
    if (!device_ok(g)) return fail(FV3_EDEVICE, "current HIP device differs from the grid's device");
    long need = fv3::noalloc_mass_doubles(g);
    long cap = (long)(FV3_NOALLOC_SCRATCH_BYTES / sizeof(double));
    if (need > cap)
        return fail(FV3_ESHAPE, "grid needs " + std::to_string(need * (long)sizeof(double)) +
                                    " bytes of block partials; the fixed scratch holds " +
                                    std::to_string((long)FV3_NOALLOC_SCRATCH_BYTES));
    fv3_status st = fv3::run_mass_sums_noalloc(g, delp, pt, q, nq, dev_out, (hipStream_t)stream);
    if (st != FV3_OK) return fail(st, "allocation-free mass sums failed");
    return FV3_OK;
}

fv3_status fv3_halo_fill(const fv3_grid *g, void *const *fields, int n_fields, int levels, int fp64,
                         void *stream)
{
    if (!g || !fields || n_fields < 1) return fail(FV3_EINVAL, "NULL argument");
    if (levels < 1 || levels > g->nz + 1) return fail(FV3_ESHAPE, "levels must be in [1, nz + 1]");
    for (int m = 0; m < n_fields; m++)
        if (!fields[m]) return fail(FV3_EINVAL, "NULL field pointer");
    return fv3::run_halo_cells(g, fields, n_fields, levels, fp64, (hipStream_t)stream);
}

fv3_status fv3_device_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst) return fail(FV3_EINVAL, "NULL pointer");
    if (bytes % 16 != 0 || ((size_t)src | (size_t)dst) % 16 != 0)
        return fail(FV3_EINVAL, "bytes and both addresses must be multiples of 16");
    const char *a = (const char *)src, *b = (const char *)dst;
    if (a < b + bytes && b < a + bytes) return fail(FV3_EINVAL, "source and destination overlap");
    return fv3::run_device_copy(src, dst, bytes, (hipStream_t)stream);
}

fv3_status fv3_timing_start(const char *filter)
{
    fv3::timing_start(filter);
    return FV3_OK;
}

int fv3_timing_stop(char *names, int names_cap, double *total_ms, long *counts, int cap)
{
    if (!names || !total_ms || !counts || cap < 1) return (int)fail(FV3_EINVAL, "NULL output");
    return fv3::timing_stop(names, names_cap, total_ms, counts, cap);
}

fv3_status fv3_check_status(const fv3_grid *g, void *stream)
{
    if (!g) return fail(FV3_EINVAL, "NULL grid");
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return fail(FV3_EDEVICE, "stream sync failed");
    int h[3] = {0, 0, 0};
    if (hipMemcpy(h, g->flags, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(FV3_EDEVICE, "flag read failed");
    int zero[3] = {0, 0, 0};
    if (hipMemcpy(g->flags, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FV3_EDEVICE, "flag reset failed");
    if (h[0]) return fail(FV3_ECFL, "a Courant number exceeded 1");
    if (h[1]) return fail(FV3_ENONFINITE, "a prognostic field became non-finite");
    if (h[2]) return fail(FV3_EREMAP, "reference interfaces do not increase in some column");
    return FV3_OK;
}

}  // extern "C"
